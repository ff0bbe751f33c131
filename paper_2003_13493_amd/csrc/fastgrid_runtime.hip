// Host runtime of libfastgrid: argument validation, contexts, the plain
// entry point, batched submission with tickets, and graph-captured resident
// batches.  See include/fastgrid.h for the contract of every entry point.
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fg_internal.h"

#define FG_API extern "C" __attribute__((visibility("default")))

static_assert(sizeof(fast_plane) == 24, "fast_plane layout is part of the ABI");
static_assert(sizeof(fast_feature) == 8, "fast_feature layout is part of the ABI");
static_assert(sizeof(fast_job) == 40, "fast_job layout is part of the ABI");
static_assert(sizeof(fast_shape_region) == 20, "fast_shape_region layout is part of the ABI");
static_assert(sizeof(fast_frontend_job) == 88, "fast_frontend_job layout is part of the ABI");

namespace {

constexpr int TICKET_RING = 256;   // submissions tracked per context
constexpr int TABLE_SLOTS = 8;     // job tables that may be in flight at once
// Default region side.  A one-frame call on a small frame switches to
// SMALL_REGION (see plain_layout).
constexpr int DEFAULT_REGION = 64;
constexpr int SMALL_REGION = 32;

// A submission's job table and work items travel in one host-to-device copy:
// the jobs at offset 0 and the items from items_offset(njobs), in a pinned
// staging buffer and its device twin of `cap` bytes.
struct TableSlot {
    uint8_t *host = nullptr;       // pinned staging buffer
    uint8_t *dev = nullptr;
    size_t cap = 0;
    unsigned *counter = nullptr;   // persistent-queue counters (FG_COUNTER_WORDS)
    uint64_t ticket = 0;           // last submission that used this slot
};

constexpr size_t items_offset(int njobs) { return (sizeof(fg_job) * (size_t)njobs + 15) & ~(size_t)15; }

struct Plan {
    bool live = false;
    fg_job *dev = nullptr;
    fg_item *items = nullptr;
    unsigned *counter = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int njobs = 0;
    int total = 0, total_upper = 0, max_levels = 0, mw1 = 0, mh1 = 0;
    bool all_single = true;
    bool launched = false;
    hipStream_t last_stream = nullptr;   // launches of a plan are ordered on one stream
};

// Device memory that enqueued work may still read when its owner is released
// (a destroyed plan, a staging buffer outgrown by a submission).  It is freed
// once `done` has completed, at the next setup call that finds it so, or when
// the context is destroyed: hipFree waits for the whole device, so it is kept
// off the launch, submit and destroy paths.
struct Retired {
    void *dev[3] = {nullptr, nullptr, nullptr};
    void *host = nullptr;                // pinned staging buffer
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;           // null: nothing enqueued reads it
};

}  // namespace

// Device scratch of fast_submit_static: the queue counters, the job table
// and the work items of one submission, in a file-scope array instead of
// memory allocated per context.  Each device holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress returns for that
// device (the array's name is a host-side stand-in, not a device address).
namespace {
constexpr size_t STATIC_COUNTER_BYTES = 2304;   // FG_COUNTER_WORDS words
constexpr size_t static_items_offset(int njobs) { return STATIC_COUNTER_BYTES + ((sizeof(fg_job) * (size_t)njobs + 15) & ~(size_t)15); }
constexpr size_t STATIC_BYTES = static_items_offset(FAST_STATIC_MAX_JOBS) + sizeof(fg_item) * FAST_STATIC_MAX_ITEMS;
static_assert(FG_COUNTER_WORDS * sizeof(unsigned) <= STATIC_COUNTER_BYTES, "counter words fit their slot");
static_assert(STATIC_COUNTER_BYTES % 256 == 0, "job table 256-byte aligned");
static_assert(STATIC_BYTES == FAST_STATIC_SCRATCH_BYTES, "the header states the scratch size");
constexpr int MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) uint8_t scratch[STATIC_BYTES];

namespace {
std::mutex g_scratch_mu;
uint8_t *g_scratch_addr[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller's DeviceGuard makes it so).
hipError_t scratch_address(int device, uint8_t **out) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = (uint8_t *)p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}
}  // namespace

struct fast_ctx {
    int device = 0;
    fg_launch launch{};
    std::string err;
    uint64_t next_ticket = 1;
    hipEvent_t events[TICKET_RING] = {};
    uint64_t event_ticket[TICKET_RING] = {};
    TableSlot slots[TABLE_SLOTS];
    std::vector<Plan> plans;
    std::vector<Retired> retired;
    hipStream_t capture_stream = nullptr;
    // the serving loops' launch streams, created on first use and kept for the
    // context's life: the ticket events of their launches stay in the event
    // ring after a loop returns, and an event must not outlive the stream it
    // was last recorded on
    hipStream_t pump_streams[FAST_PUMP_MAX_LANES] = {};
    // tuned region sides of one-frame calls, per frame shape (fast_set_shape_table)
    std::vector<fast_shape_region> shapes;
    // fast_submit_static: the device scratch address, a pinned staging buffer
    // of STATIC_BYTES set up at creation, and the event that marks the last
    // table copy out of it
    uint8_t *static_dev = nullptr;
    uint8_t *static_host = nullptr;
    hipEvent_t static_copied = nullptr;
    bool static_pending = false;
};

namespace {

int fail(fast_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

// Region layout of a one-frame call.  With an explicit side (plain_region
// != 0) that side; else the tuned side of the frame's shape, if the shape
// table has one; otherwise the batch side, unless the frame has fewer
// regions than half the CUs and at most 3 levels: then 32-pixel regions give
// 4x the workgroups at a still moderate halo cost (MI355X, 256 threads:
// 640x480 L=3 10.8 us against 17.7 us; 1280x720, 240 regions, 16.6 against
// 15.0 us; 1920x1080 L=4 42.5 against 24.5 us).
void plain_layout(const fast_ctx *c, fg_job &j) {
    fg_launch L = c->launch;
    if (L.plain_region) {
        L.region = L.plain_region;
        fg_job_layout(j, L);
        return;
    }
    // a tuned side for this frame shape
    for (const fast_shape_region &e : c->shapes) {
        if (e.width == j.w[0] && e.height == j.h[0] && e.levels == j.levels && e.cell == j.cell) {
            L.region = e.region;
            fg_job_layout(j, L);
            return;
        }
    }
    fg_job_layout(j, L);
    if (j.levels <= 3 && j.rx * j.ry * 2 < L.num_cu) {
        L.region = SMALL_REGION;
        fg_job_layout(j, L);
    }
}

int hip_fail(fast_ctx *c, hipError_t e, const char *what) {
    if (c) c->err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return FAST_EHIP;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool plane_ok(const fast_plane &p, std::string &why) {
    if (!p.data) { why = "plane data is NULL"; return false; }
    if (((uintptr_t)p.data & 15u) != 0) { why = "plane data not 16-byte aligned"; return false; }
    if (p.width < 1 || p.height < 1) { why = "plane has zero size"; return false; }
    if (p.width > 65535 || p.height > 65535) { why = "plane larger than 65535"; return false; }
    if (p.pitch < p.width) { why = "pitch < width"; return false; }
    if (p.pitch % 16 != 0) { why = "pitch not a multiple of 16"; return false; }
    return true;
}

int check_pyr(fast_ctx *c, const fast_plane *pyr, int levels) {
    if (!pyr) return fail(c, FAST_EINVAL, "pyr is NULL");
    if (levels < 1 || levels > FAST_MAX_LEVELS) return fail(c, FAST_EINVAL, "levels not in 1..8");
    std::string why;
    for (int k = 0; k < levels; ++k) {
        if (!plane_ok(pyr[k], why)) return fail(c, FAST_EINVAL, "level " + std::to_string(k) + ": " + why);
        if (k > 0 && (pyr[k].width != pyr[k - 1].width / 2 || pyr[k].height != pyr[k - 1].height / 2))
            return fail(c, FAST_EINVAL, "level " + std::to_string(k) + " is not the floor half of level " +
                                            std::to_string(k - 1));
    }
    return FAST_OK;
}

int check_params(fast_ctx *c, int levels, int t, int n, int cell) {
    if (t < 0 || t > 255) return fail(c, FAST_EINVAL, "t not in 0..255");
    if (n < 1 || n > 16) return fail(c, FAST_EINVAL, "n not in 1..16");
    if (cell < 1 || cell > FAST_MAX_CELL) return fail(c, FAST_EINVAL, "cell not in 1..256");
    if (cell % (1 << (levels - 1)) != 0) return fail(c, FAST_EINVAL, "cell not a multiple of 2^(levels-1)");
    return FAST_OK;
}

int make_job(fast_ctx *c, const fast_plane *pyr, int levels, int t, int n, int cell, int score,
             fast_feature *out, fg_job &j, bool need_out = true, bool plain = false) {
    int rc = check_pyr(c, pyr, levels);
    if (rc) return rc;
    rc = check_params(c, levels, t, n, cell);
    if (rc) return rc;
    if (score < FAST_SCORE_SADB || score > FAST_SCORE_MT) return fail(c, FAST_EINVAL, "unknown score kind");
    if (!out && need_out) return fail(c, FAST_EINVAL, "out is NULL");
    memset(&j, 0, sizeof(j));
    for (int k = 0; k < levels; ++k) {
        j.lvl[k] = pyr[k].data;
        j.w[k] = pyr[k].width;
        j.h[k] = pyr[k].height;
        j.pitch[k] = pyr[k].pitch;
    }
    j.levels = levels;
    j.t = t;
    j.n = n;
    j.cell = cell;
    j.score = score;
    j.out = out;
    if (plain) plain_layout(c, j);
    else fg_job_layout(j, c->launch);
    return FAST_OK;
}

// Record the completion event of a new submission; returns its ticket.
int record_ticket(fast_ctx *c, hipStream_t s, uint64_t *ticket) {
    const uint64_t tk = c->next_ticket;
    const int i = (int)(tk % TICKET_RING);
    if (c->event_ticket[i] != 0) {
        // recycle: the previous holder of this event must be finished
        hipError_t e = hipEventSynchronize(c->events[i]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    }
    hipError_t e = hipEventRecord(c->events[i], s);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord");
    c->event_ticket[i] = tk;
    c->next_ticket = tk + 1;
    if (ticket) *ticket = tk;
    return FAST_OK;
}

// Queue device memory for release once the work enqueued on `s` so far has
// completed (s may be null when no work reads it).
int retire(fast_ctx *c, Retired r, bool enqueued, hipStream_t s) {
    if (enqueued) {
        hipError_t e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r.done, s);
        if (e != hipSuccess) return hip_fail(c, e, "retire event");
    }
    c->retired.push_back(r);
    return FAST_OK;
}

void release(Retired &r) {
    if (r.exec) (void)hipGraphExecDestroy(r.exec);
    if (r.graph) (void)hipGraphDestroy(r.graph);
    for (void *p : r.dev)
        if (p) (void)hipFree(p);
    if (r.host) (void)hipHostFree(r.host);
    if (r.done) (void)hipEventDestroy(r.done);
    r = Retired();
}

// Free retired memory whose readers have finished (setup calls only: hipFree
// synchronises the device).  wait: block until every reader has finished.
void reap(fast_ctx *c, bool wait) {
    std::vector<Retired> keep;
    for (Retired &r : c->retired) {
        bool finished = !r.done;
        if (!finished && wait) {
            (void)hipEventSynchronize(r.done);
            finished = true;
        } else if (!finished) {
            finished = hipEventQuery(r.done) != hipErrorNotReady;
        }
        if (finished) release(r);
        else keep.push_back(r);
    }
    c->retired.swap(keep);
}

// 1 done, 0 pending, <0 error.
int ticket_state(fast_ctx *c, uint64_t tk) {
    if (tk == 0 || tk >= c->next_ticket) return fail(c, FAST_EINVAL, "unknown ticket");
    if (c->event_ticket[tk % TICKET_RING] != tk)
        return 1;   // its event was recycled, which only happens after it completed
    hipError_t e = hipEventQuery(c->events[tk % TICKET_RING]);
    if (e == hipSuccess) {
        // seen complete: the ring entry is free, so recycling it later needs
        // no wait on an event whose stream may be gone by then
        c->event_ticket[tk % TICKET_RING] = 0;
        return 1;
    }
    if (e == hipErrorNotReady) return 0;
    return hip_fail(c, e, "hipEventQuery");
}

int build_table(fast_ctx *c, const fast_job *jobs, int njobs, fg_job *table, int &total, int &total_upper,
                int &max_levels, int &max_w1, int &max_h1, bool &all_single) {
    if (!jobs) return fail(c, FAST_EINVAL, "jobs is NULL");
    if (njobs < 1 || njobs > FAST_MAX_JOBS) return fail(c, FAST_EINVAL, "njobs not in 1..4096");
    total = 0;
    total_upper = 0;
    all_single = true;
    max_levels = 1;
    max_w1 = 1;
    max_h1 = 1;
    for (int i = 0; i < njobs; ++i) {
        const fast_job &q = jobs[i];
        int rc = make_job(c, q.pyr, q.levels, q.t, q.n, q.cell, q.score, q.out, table[i]);
        if (rc) {
            c->err = "job " + std::to_string(i) + ": " + c->err;
            return rc;
        }
        table[i].region_base = total;
        total += table[i].rx * table[i].ry;
        if (q.levels > FG_MAX_FUSED) total_upper += table[i].rx * table[i].ry;
        if (table[i].rcells * table[i].cell > FG_SUB) all_single = false;
        if (q.levels > max_levels) max_levels = q.levels;
        if (q.levels > 1) {
            if (table[i].w[1] > max_w1) max_w1 = table[i].w[1];
            if (table[i].h[1] > max_h1) max_h1 = table[i].h[1];
        }
    }
    return FAST_OK;
}

// The work items (job, region) of a batch.  Whole regions come first and the
// regions clipped at a frame's right or bottom edge last, each group in job
// and region order: the cheap items end the queue, so the persistent
// workgroups run out of work closer together.
// The regions of the jobs with more than FG_MAX_FUSED levels follow, in job
// and region order, for the pass over their deeper levels.
void fill_items(const fg_job *table, int njobs, fg_item *items) {
    int n = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < njobs; ++j) {
            const fg_job &J = table[j];
            const int side = J.rcells * J.cell;
            for (int r = 0; r < J.rx * J.ry; ++r) {
                const int x0 = (r % J.rx) * side, y0 = (r / J.rx) * side;
                const bool whole = x0 + side <= J.w[0] && y0 + side <= J.h[0];
                if (whole == (pass == 0)) items[n++] = fg_item{(uint32_t)j, (uint32_t)r};
            }
        }
    }
    for (int j = 0; j < njobs; ++j)
        if (table[j].levels > FG_MAX_FUSED)
            for (int r = 0; r < table[j].rx * table[j].ry; ++r) items[n++] = fg_item{(uint32_t)j, (uint32_t)r};
}

}  // namespace

FG_API const char *fast_strerror(int status) {
    switch (status) {
        case FAST_OK: return "success";
        case FAST_EINVAL: return "invalid argument";
        case FAST_ENOMEM: return "out of memory";
        case FAST_EHIP: return "HIP runtime error";
        case FAST_EBUSY: return "all in-flight slots busy";
        case FAST_ETIMEDOUT: return "timed out";
        default: return "unknown status";
    }
}

FG_API const char *fast_last_error(const fast_ctx *c) { return c ? c->err.c_str() : "no context"; }

// Staging buffers of a submission slot, `cap` bytes each, and its queue
// counters (zeroed).
int slot_alloc(fast_ctx *c, TableSlot &S, size_t cap) {
    hipError_t e = hipHostMalloc((void **)&S.host, cap, hipHostMallocDefault);
    if (e != hipSuccess) { S.host = nullptr; return hip_fail(c, e, "hipHostMalloc job table"); }
    e = hipMalloc((void **)&S.dev, cap);
    if (e != hipSuccess) { S.dev = nullptr; return hip_fail(c, e, "hipMalloc job table"); }
    S.cap = cap;
    if (!S.counter) {
        e = hipMalloc((void **)&S.counter, FG_COUNTER_WORDS * sizeof(unsigned));
        if (e != hipSuccess) { S.counter = nullptr; return hip_fail(c, e, "hipMalloc counter"); }
        e = hipMemset(S.counter, 0, FG_COUNTER_WORDS * sizeof(unsigned));
        if (e != hipSuccess) return hip_fail(c, e, "hipMemset counter");
    }
    return FAST_OK;
}

// Default staging capacity of a slot: FAST_MAX_JOBS jobs and 65536 work items.
size_t slot_default_cap() { return items_offset(FAST_MAX_JOBS) + sizeof(fg_item) * 65536; }

FG_API int fast_ctx_create(int hip_device, fast_ctx **out) {
    if (!out) return FAST_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return FAST_EINVAL;
    fast_ctx *c = new (std::nothrow) fast_ctx();
    if (!c) return FAST_ENOMEM;
    c->device = hip_device;
    DeviceGuard g(hip_device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess || cus < 1)
        cus = 256;
    c->launch.num_cu = cus;
    c->launch.region = DEFAULT_REGION;
    c->launch.plain_region = 0;
    c->launch.block = 256;
    c->launch.blocks_per_cu = 3;
    for (int i = 0; i < TICKET_RING; ++i) {
        hipError_t e = hipEventCreateWithFlags(&c->events[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            fast_ctx_destroy(c);
            return FAST_EHIP;
        }
    }
    // every submission slot is ready before the first submit, so fast_submit
    // allocates nothing (unless a submission outgrows a slot)
    for (auto &S : c->slots) {
        if (slot_alloc(c, S, slot_default_cap()) != FAST_OK) {
            const int rc = FAST_ENOMEM;
            fast_ctx_destroy(c);
            return rc;
        }
    }
    // the scratch array of fast_submit_static: its device address, looked up
    // once per device, and the pinned buffer its tables are staged in
    uint8_t *dev_scratch = nullptr;
    hipError_t se = scratch_address(hip_device, &dev_scratch);
    if (se == hipSuccess) se = hipHostMalloc((void **)&c->static_host, STATIC_BYTES, hipHostMallocDefault);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&c->static_copied, hipEventDisableTiming);
    if (se != hipSuccess) {
        fast_ctx_destroy(c);
        return FAST_EHIP;
    }
    c->static_dev = dev_scratch;
    *out = c;
    return FAST_OK;
}

FG_API void fast_ctx_destroy(fast_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    // wait for this context's own work: its outstanding submissions, the
    // launches of its live plans and the readers of retired memory (the frees
    // below then find the device idle as far as this context is concerned)
    for (int i = 0; i < TICKET_RING; ++i)
        if (c->events[i] && c->event_ticket[i]) (void)hipEventSynchronize(c->events[i]);
    // a live plan records no event per launch; its stream may be gone by now,
    // so its launches are waited for with the device (the frees below would
    // wait for the device anyway)
    bool plan_pending = false;
    for (auto &p : c->plans) plan_pending = plan_pending || (p.live && p.launched);
    if (plan_pending) (void)hipDeviceSynchronize();
    reap(c, true);
    for (auto &p : c->plans) {
        if (p.exec) (void)hipGraphExecDestroy(p.exec);
        if (p.graph) (void)hipGraphDestroy(p.graph);
        if (p.dev) (void)hipFree(p.dev);
        if (p.items) (void)hipFree(p.items);
        if (p.counter) (void)hipFree(p.counter);
    }
    for (auto &s : c->slots) {
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.counter) (void)hipFree(s.counter);
    }
    if (c->static_copied) {
        if (c->static_pending) (void)hipEventSynchronize(c->static_copied);
        (void)hipEventDestroy(c->static_copied);
    }
    if (c->static_host) (void)hipHostFree(c->static_host);
    for (auto &e : c->events)
        if (e) (void)hipEventDestroy(e);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (hipStream_t s : c->pump_streams)
        if (s) (void)hipStreamDestroy(s);
    delete c;
}

FG_API int fast_pyr_dims(int width, int height, int levels, fast_plane *dims) {
    if (!dims || levels < 1 || levels > FAST_MAX_LEVELS || width < 1 || height < 1 || width > 65535 ||
        height > 65535)
        return FAST_EINVAL;
    int w = width, h = height;
    for (int k = 0; k < levels; ++k) {
        if (w < 1 || h < 1) return FAST_EINVAL;
        dims[k].data = nullptr;
        dims[k].width = w;
        dims[k].height = h;
        dims[k].pitch = (w + 63) / 64 * 64;
        w /= 2;
        h /= 2;
    }
    return FAST_OK;
}

FG_API int fast_grid_dims(int width, int height, int cell, int *gw, int *gh) {
    if (!gw || !gh || width < 1 || height < 1 || cell < 1) return FAST_EINVAL;
    *gw = (width + cell - 1) / cell;
    *gh = (height + cell - 1) / cell;
    return FAST_OK;
}

FG_API int fast_set_launch(fast_ctx *c, int region, int block, int bpc) {
    if (!c) return FAST_EINVAL;
    if (region != 0 && (region < 16 || region > 256)) return fail(c, FAST_EINVAL, "region not 0 or in 16..256");
    if (block < 64 || block > 512 || block % 64 != 0)
        return fail(c, FAST_EINVAL, "block not a multiple of 64 in 64..512");
    if (bpc < 1 || bpc > 16) return fail(c, FAST_EINVAL, "blocks per CU not in 1..16");
    c->launch.region = region ? region : DEFAULT_REGION;
    c->launch.plain_region = region;
    c->launch.block = block;
    c->launch.blocks_per_cu = bpc;
    return FAST_OK;
}

FG_API int fast_set_shape_table(fast_ctx *c, const fast_shape_region *entries, int n) {
    if (!c) return FAST_EINVAL;
    if (n < 0 || n > FAST_MAX_SHAPES) return fail(c, FAST_EINVAL, "n not in 0..FAST_MAX_SHAPES");
    if (n > 0 && !entries) return fail(c, FAST_EINVAL, "entries is NULL");
    std::vector<fast_shape_region> table;
    for (int i = 0; i < n; ++i) {
        const fast_shape_region &e = entries[i];
        const std::string at = "entry " + std::to_string(i) + ": ";
        if (e.width < 1 || e.height < 1 || e.width > 65535 || e.height > 65535)
            return fail(c, FAST_EINVAL, at + "width or height not in 1..65535");
        if (e.levels < 1 || e.levels > FAST_MAX_LEVELS) return fail(c, FAST_EINVAL, at + "levels not in 1..8");
        if ((e.width >> (e.levels - 1)) < 1 || (e.height >> (e.levels - 1)) < 1)
            return fail(c, FAST_EINVAL, at + "a level of size 0");
        if (check_params(c, e.levels, 0, 1, e.cell) != FAST_OK) return fail(c, FAST_EINVAL, at + c->err);
        if (e.region < 16 || e.region > 256) return fail(c, FAST_EINVAL, at + "region not in 16..256");
        for (const fast_shape_region &f : table)
            if (f.width == e.width && f.height == e.height && f.levels == e.levels && f.cell == e.cell)
                return fail(c, FAST_EINVAL, at + "shape listed twice");
        table.push_back(e);
    }
    c->shapes.swap(table);
    return FAST_OK;
}

FG_API int fast_shape_region_of(fast_ctx *c, int width, int height, int levels, int cell, int *region) {
    if (!c) return FAST_EINVAL;
    if (!region) return fail(c, FAST_EINVAL, "region is NULL");
    if (width < 1 || height < 1 || width > 65535 || height > 65535)
        return fail(c, FAST_EINVAL, "width or height not in 1..65535");
    if (levels < 1 || levels > FAST_MAX_LEVELS) return fail(c, FAST_EINVAL, "levels not in 1..8");
    int rc = check_params(c, levels, 0, 1, cell);
    if (rc) return rc;
    fg_job j;
    memset(&j, 0, sizeof(j));
    j.w[0] = width;
    j.h[0] = height;
    j.levels = levels;
    j.cell = cell;
    plain_layout(c, j);
    *region = j.rcells * cell;
    return FAST_OK;
}

FG_API int fast_pyr_build(fast_ctx *c, const fast_plane *pyr, int levels, void *stream) {
    if (!c) return FAST_EINVAL;
    int rc = check_pyr(c, pyr, levels);
    if (rc) return rc;
    fg_job j;
    memset(&j, 0, sizeof(j));
    for (int k = 0; k < levels; ++k) {
        j.lvl[k] = pyr[k].data;
        j.w[k] = pyr[k].width;
        j.h[k] = pyr[k].height;
        j.pitch[k] = pyr[k].pitch;
    }
    j.levels = levels;
    DeviceGuard g(c->device);
    hipError_t e = fg_launch_pyramid(j, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pyramid launch");
    return FAST_OK;
}

FG_API int fast_detect_grid(fast_ctx *c, const fast_plane *pyr, int levels, int t, int n, int cell,
                            fast_feature *out, void *stream) {
    return fast_detect_grid_score(c, pyr, levels, t, n, cell, FAST_SCORE_SADB, out, stream);
}

FG_API int fast_detect_grid_score(fast_ctx *c, const fast_plane *pyr, int levels, int t, int n, int cell,
                                  int score, fast_feature *out, void *stream) {
    if (!c) return FAST_EINVAL;
    fg_job j;
    int rc = make_job(c, pyr, levels, t, n, cell, score, out, j, true, true);
    if (rc) return rc;
    DeviceGuard g(c->device);
    hipError_t e = fg_launch_plain(j, c->launch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "detect launch");
    return FAST_OK;
}

// Score maps of levels 0..levels-1 with floor-halved sizes of width x height.
int check_maps(fast_ctx *c, uint16_t *const *maps, const int32_t *pitch, int width, int height, int levels) {
    if (!maps || !pitch) return fail(c, FAST_EINVAL, "maps or map_pitch is NULL");
    int w = width, h = height;
    for (int k = 0; k < levels; ++k) {
        if (w < 1 || h < 1) return fail(c, FAST_EINVAL, "level " + std::to_string(k) + " has zero size");
        if (!maps[k]) return fail(c, FAST_EINVAL, "map " + std::to_string(k) + " is NULL");
        if (((uintptr_t)maps[k] & 1u) != 0) return fail(c, FAST_EINVAL, "map not 2-byte aligned");
        if (pitch[k] < w) return fail(c, FAST_EINVAL, "map pitch < level width");
        w >>= 1;
        h >>= 1;
    }
    return FAST_OK;
}

FG_API int fast_score_maps(fast_ctx *c, const fast_plane *pyr, int levels, int t, int n, int score,
                           uint16_t *const *maps, const int32_t *map_pitch, void *stream) {
    if (!c) return FAST_EINVAL;
    fg_job j;
    // any valid cell: it only shapes the work decomposition here
    int rc = make_job(c, pyr, levels, t, n, 1 << (levels - 1 < 4 ? 4 : levels - 1), score, nullptr, j, false, true);
    if (rc) return rc;
    rc = check_maps(c, maps, map_pitch, pyr[0].width, pyr[0].height, levels);
    if (rc) return rc;
    for (int k = 0; k < levels; ++k) {
        j.smap[k] = maps[k];
        j.smap_pitch[k] = map_pitch[k];
    }
    DeviceGuard g(c->device);
    hipError_t e = fg_launch_score_maps(j, c->launch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "score map launch");
    return FAST_OK;
}

FG_API int fast_nms_grid(fast_ctx *c, uint16_t *const *maps, const int32_t *map_pitch, int width, int height,
                         int levels, int radius, int cell, fast_feature *out, void *stream) {
    if (!c) return FAST_EINVAL;
    if (levels < 1 || levels > FAST_MAX_LEVELS) return fail(c, FAST_EINVAL, "levels not in 1..8");
    if (width < 1 || height < 1 || width > 65535 || height > 65535)
        return fail(c, FAST_EINVAL, "width or height not in 1..65535");
    if (radius < 1 || radius > 4) return fail(c, FAST_EINVAL, "radius not in 1..4");
    int rc = check_params(c, levels, 0, 1, cell);
    if (rc) return rc;
    if (!out) return fail(c, FAST_EINVAL, "out is NULL");
    rc = check_maps(c, maps, map_pitch, width, height, levels);
    if (rc) return rc;
    fg_job j;
    memset(&j, 0, sizeof(j));
    int w = width, h = height;
    for (int k = 0; k < levels; ++k) {
        j.w[k] = w;
        j.h[k] = h;
        j.smap[k] = maps[k];
        j.smap_pitch[k] = map_pitch[k];
        w >>= 1;
        h >>= 1;
    }
    j.levels = levels;
    j.cell = cell;
    j.out = out;
    plain_layout(c, j);
    DeviceGuard g(c->device);
    hipError_t e = fg_launch_nms_grid(j, radius, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "nms launch");
    return FAST_OK;
}

FG_API int fast_track(fast_ctx *c, const fast_plane *tpl, const fast_plane *img, int levels, const float *feats,
                      float *q, int32_t *status, int32_t *iters, int nfeat, int mode, int max_iter, float eps,
                      void *stream) {
    if (!c) return FAST_EINVAL;
    int rc = check_pyr(c, tpl, levels);
    if (rc) return rc;
    rc = check_pyr(c, img, levels);
    if (rc) return rc;
    if (tpl[0].width != img[0].width || tpl[0].height != img[0].height)
        return fail(c, FAST_EINVAL, "template and image sizes differ");
    if (mode & ~(FAST_TRACK_GAIN | FAST_TRACK_OFFSET)) return fail(c, FAST_EINVAL, "unknown mode bits");
    if (max_iter < 0 || max_iter > 1000) return fail(c, FAST_EINVAL, "max_iter not in 0..1000");
    if (!(eps >= 0.0f) || eps > 1e30f) return fail(c, FAST_EINVAL, "eps not a finite value >= 0");
    if (nfeat < 0 || nfeat > (1 << 24)) return fail(c, FAST_EINVAL, "nfeat not in 0..2^24");
    if (nfeat > 0 && (!feats || !q || !status)) return fail(c, FAST_EINVAL, "feats, q or status is NULL");
    if ((((uintptr_t)feats | (uintptr_t)q | (uintptr_t)status | (uintptr_t)iters) & 3u) != 0)
        return fail(c, FAST_EINVAL, "feats, q, status or iters not 4-byte aligned");
    fg_track_args A;
    memset(&A, 0, sizeof(A));
    for (int k = 0; k < levels; ++k) {
        A.tpl[k] = tpl[k].data;
        A.img[k] = img[k].data;
        A.w[k] = tpl[k].width;
        A.h[k] = tpl[k].height;
        A.tpitch[k] = tpl[k].pitch;
        A.ipitch[k] = img[k].pitch;
    }
    A.levels = levels;
    A.feats = feats;
    A.q = q;
    A.status = status;
    A.iters = iters;
    A.nfeat = nfeat;
    A.mode = mode;
    A.max_iter = max_iter;
    A.eps = eps;
    DeviceGuard g(c->device);
    hipError_t e = fg_launch_track(A, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "track launch");
    return FAST_OK;
}

FG_API int fast_submit(fast_ctx *c, const fast_job *jobs, int njobs, void *stream, uint64_t *ticket) {
    if (!c) return FAST_EINVAL;
    if (!ticket) return fail(c, FAST_EINVAL, "ticket is NULL");
    // pick a table slot whose last submission has finished
    int slot = -1;
    for (int i = 0; i < TABLE_SLOTS && slot < 0; ++i) {
        const uint64_t tk = c->slots[i].ticket;
        if (tk == 0) slot = i;
        else {
            int st = ticket_state(c, tk);
            if (st < 0) return st;
            if (st == 1) slot = i;
        }
    }
    if (slot < 0) return fail(c, FAST_EBUSY, "all job tables are in flight");
    DeviceGuard g(c->device);
    TableSlot &S = c->slots[slot];
    int total, total_upper, max_levels, mw1, mh1;
    bool all_single;
    // the staging buffer always has room for FAST_MAX_JOBS jobs
    int rc = build_table(c, jobs, njobs, (fg_job *)S.host, total, total_upper, max_levels, mw1, mh1, all_single);
    if (rc) return rc;
    const int nitems = total + total_upper;
    const size_t off = items_offset(njobs), bytes = off + sizeof(fg_item) * (size_t)nitems;
    if (bytes > S.cap) {
        // the slot is idle (its last submission has finished), so nothing
        // reads its old buffers; they are released at the next setup call
        // rather than here, since hipFree would wait for the whole device
        TableSlot grown;
        grown.counter = S.counter;
        int arc = slot_alloc(c, grown, std::max(bytes, slot_default_cap()));
        if (arc != FAST_OK) {
            if (grown.host) (void)hipHostFree(grown.host);
            return arc;
        }
        memcpy(grown.host, S.host, off);
        Retired r;
        r.dev[0] = S.dev;
        r.host = S.host;
        arc = retire(c, r, false, nullptr);
        if (arc != FAST_OK) return arc;
        grown.ticket = S.ticket;
        S = grown;
    }
    const fg_job *jobs_dev = (const fg_job *)S.dev;
    const fg_item *items_dev = (const fg_item *)(S.dev + off);
    fill_items((const fg_job *)S.host, njobs, (fg_item *)(S.host + off));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(S.dev, S.host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "job table upload");
    e = fg_launch_batch(jobs_dev, items_dev, njobs, total, total_upper, max_levels, mw1, mh1, all_single,
                        S.counter, c->launch, s);
    if (e != hipSuccess) return hip_fail(c, e, "batch launch");
    rc = record_ticket(c, s, ticket);
    if (rc) return rc;
    S.ticket = *ticket;
    return FAST_OK;
}

FG_API int fast_submit_static(fast_ctx *c, const fast_job *jobs, int njobs, void *stream, uint64_t *ticket) {
    if (!c) return FAST_EINVAL;
    if (!jobs) return fail(c, FAST_EINVAL, "jobs is NULL");
    if (njobs < 1 || njobs > FAST_STATIC_MAX_JOBS)
        return fail(c, FAST_EINVAL, "njobs not in 1.." + std::to_string(FAST_STATIC_MAX_JOBS) +
                                        " (the static scratch limit)");
    if (!c->static_dev || !c->static_host) return fail(c, FAST_EINVAL, "context has no static scratch");
    DeviceGuard g(c->device);
    // the staging buffer is reused: the previous call's copy out of it must
    // have run before it is rewritten
    if (c->static_pending) {
        const hipError_t e = hipEventSynchronize(c->static_copied);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize (static staging)");
        c->static_pending = false;
    }
    uint8_t *host = c->static_host;
    int total, total_upper, max_levels, mw1, mh1;
    bool all_single;
    int rc = build_table(c, jobs, njobs, (fg_job *)(host + STATIC_COUNTER_BYTES), total, total_upper, max_levels,
                         mw1, mh1, all_single);
    if (rc) return rc;
    const int nitems = total + total_upper;
    if (nitems > FAST_STATIC_MAX_ITEMS)
        return fail(c, FAST_EINVAL, "the jobs need " + std::to_string(nitems) + " work items, more than the " +
                                        std::to_string(FAST_STATIC_MAX_ITEMS) + " the static scratch holds");
    const size_t off = static_items_offset(njobs), bytes = off + sizeof(fg_item) * (size_t)nitems;
    // the queue counters travel with the table, so they start at zero whatever
    // an earlier call left in the scratch
    memset(host, 0, STATIC_COUNTER_BYTES);
    fill_items((const fg_job *)(host + STATIC_COUNTER_BYTES), njobs, (fg_item *)(host + off));
    hipStream_t s = (hipStream_t)stream;
    uint8_t *dev = c->static_dev;
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "static table upload");
    e = hipEventRecord(c->static_copied, s);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventRecord (static staging)");
    c->static_pending = true;
    e = fg_launch_batch((const fg_job *)(dev + STATIC_COUNTER_BYTES), (const fg_item *)(dev + off), njobs, total,
                        total_upper, max_levels, mw1, mh1, all_single, (unsigned *)dev, c->launch, s);
    if (e != hipSuccess) return hip_fail(c, e, "batch launch (static)");
    if (!ticket) return FAST_OK;
    return record_ticket(c, s, ticket);
}

// Track arguments of one pyramid pair (tpl, img) for tracking kernels.
void fill_track_planes(fg_track_args &A, const fast_plane *tpl, const fast_plane *img, int levels) {
    for (int k = 0; k < levels; ++k) {
        A.tpl[k] = tpl[k].data;
        A.img[k] = img[k].data;
        A.w[k] = tpl[k].width;
        A.h[k] = tpl[k].height;
        A.tpitch[k] = tpl[k].pitch;
        A.ipitch[k] = img[k].pitch;
    }
    A.levels = levels;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

int check_track_params(fast_ctx *c, int mode, int max_iter, float eps) {
    if (mode & ~(FAST_TRACK_GAIN | FAST_TRACK_OFFSET)) return fail(c, FAST_EINVAL, "unknown mode bits");
    if (max_iter < 0 || max_iter > 1000) return fail(c, FAST_EINVAL, "max_iter not in 0..1000");
    if (!(eps >= 0.0f) || eps > 1e30f) return fail(c, FAST_EINVAL, "eps not a finite value >= 0");
    return FAST_OK;
}

// A free submission slot (its last submission has finished), or -1.
int free_slot(fast_ctx *c, int &slot) {
    slot = -1;
    for (int i = 0; i < TABLE_SLOTS && slot < 0; ++i) {
        const uint64_t tk = c->slots[i].ticket;
        if (tk == 0) slot = i;
        else {
            const int st = ticket_state(c, tk);
            if (st < 0) return st;
            if (st == 1) slot = i;
        }
    }
    return FAST_OK;
}

FG_API int fast_frontend_step(fast_ctx *c, const fast_frontend_job *jobs, int njobs, int mode, int max_iter,
                              float eps, void *stream, uint64_t *ticket) {
    if (!c) return FAST_EINVAL;
    if (!jobs) return fail(c, FAST_EINVAL, "jobs is NULL");
    if (njobs < 1 || njobs > FAST_MAX_JOBS) return fail(c, FAST_EINVAL, "njobs not in 1..4096");
    int rc = check_track_params(c, mode, max_iter, eps);
    if (rc) return rc;
    int slot;
    rc = free_slot(c, slot);
    if (rc) return rc;
    if (slot < 0) return fail(c, FAST_EBUSY, "all job tables are in flight");
    TableSlot &S = c->slots[slot];
    static_assert(sizeof(fg_fe_job) * FAST_MAX_JOBS <= items_offset(FAST_MAX_JOBS) + sizeof(fg_item) * 65536,
                  "a slot's default staging holds FAST_MAX_JOBS front-end jobs");
    fg_fe_job *table = (fg_fe_job *)S.host;
    int total_slots = 0;
    for (int i = 0; i < njobs; ++i) {
        const fast_frontend_job &q = jobs[i];
        const std::string at = "job " + std::to_string(i) + ": ";
        rc = check_pyr(c, q.cur, q.levels);
        if (rc) return fail(c, rc, at + c->err);
        if (q.prev) {
            rc = check_pyr(c, q.prev, q.levels);
            if (rc) return fail(c, rc, at + c->err);
            if (q.prev[0].width != q.cur[0].width || q.prev[0].height != q.cur[0].height)
                return fail(c, FAST_EINVAL, at + "previous and current sizes differ");
        }
        rc = check_params(c, q.levels, 0, 1, q.cell);
        if (rc) return fail(c, rc, at + c->err);
        const long gw = (q.cur[0].width + q.cell - 1) / q.cell, gh = (q.cur[0].height + q.cell - 1) / q.cell;
        if (gw * gh > FAST_MAX_GRID_CELLS) return fail(c, FAST_EINVAL, at + "more than FAST_MAX_GRID_CELLS cells");
        if (!q.slots || !q.feats || !q.count || !q.q || !q.status || !q.info)
            return fail(c, FAST_EINVAL, at + "a device array is NULL");
        if (((uintptr_t)q.slots & 7u) || !aligned4(q.feats) || !aligned4(q.count) || !aligned4(q.q) ||
            !aligned4(q.status) || !aligned4(q.info))
            return fail(c, FAST_EINVAL, at + "a device array is misaligned");
        if (q.capacity < 1 || q.capacity > FAST_MAX_TRACKS)
            return fail(c, FAST_EINVAL, at + "capacity not in 1..FAST_MAX_TRACKS");
        if (q.redetect_below < 0 || q.redetect_below > q.capacity)
            return fail(c, FAST_EINVAL, at + "redetect_below not in 0..capacity");
        fg_fe_job &J = table[i];
        memset(&J, 0, sizeof(J));
        fill_track_planes(J.A, q.prev ? q.prev : q.cur, q.cur, q.levels);
        J.A.feats = q.feats;
        J.A.q = q.q;
        J.A.status = q.status;
        J.A.iters = nullptr;
        J.A.nfeat = 0;
        J.A.mode = mode;
        J.A.max_iter = max_iter;
        J.A.eps = eps;
        J.slots = q.slots;
        J.count = q.count;
        J.info = q.info;
        J.cell = q.cell;
        J.gw = (int32_t)gw;
        J.gh = (int32_t)gh;
        J.capacity = q.capacity;
        J.redetect_below = q.redetect_below;
        J.has_prev = q.prev ? 1 : 0;
        J.feat_base = total_slots;
        total_slots += q.capacity;
    }
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = sizeof(fg_fe_job) * (size_t)njobs;
    hipError_t e = hipMemcpyAsync(S.dev, S.host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "front-end table upload");
    e = fg_launch_frontend((const fg_fe_job *)S.dev, njobs, total_slots, s);
    if (e != hipSuccess) return hip_fail(c, e, "front-end launch");
    uint64_t tk = 0;
    rc = record_ticket(c, s, &tk);
    if (rc) return rc;
    S.ticket = tk;
    if (ticket) *ticket = tk;
    return FAST_OK;
}

// ---------------------------------------------------------------------------
// Native serving loop: replay arrivals by the host clock, batch the oldest
// arrived frames whose stream has a free result slot onto free launch lanes,
// and record when each launch is seen complete.

namespace {

struct PumpLane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<int> reqs;   // requests of the launch in flight
    bool busy = false;
};

struct PumpSlots {
    std::vector<std::vector<fast_plane>> planes;   // per slot: levels planes, [0] set per request
    std::vector<char> busy;
    size_t out_bytes = 0;
};

static_assert(sizeof(fast_pump_stream) == 64 && sizeof(fast_pump_request) == 16 && sizeof(fast_pump_frontend) == 72,
              "pump ABI layout");

int pump_check(fast_ctx *c, const fast_pump_stream *streams, int nstreams, const fast_pump_request *reqs,
               int nreq) {
    for (int i = 0; i < nstreams; ++i) {
        const fast_pump_stream &S = streams[i];
        if (S.levels < 1 || S.levels > FAST_MAX_LEVELS || S.pool_frames < 1 || !S.pool || S.slots < 1 ||
            S.slots > 4096)
            return fail(c, FAST_EINVAL, "pump stream " + std::to_string(i) + " is malformed");
    }
    double last = 0.0;
    for (int r = 0; r < nreq; ++r) {
        const fast_pump_request &q = reqs[r];
        if (q.stream < 0 || q.stream >= nstreams || q.frame < 0)
            return fail(c, FAST_EINVAL, "pump request " + std::to_string(r) + " names no stream or frame");
        if (!(q.arrival_s >= last) || !(q.arrival_s < 1e9))
            return fail(c, FAST_EINVAL, "pump arrivals must be finite and non-decreasing");
        last = q.arrival_s;
    }
    return FAST_OK;
}

}  // namespace

// The loop shared by both entry points.  `slots_of(i)` is stream i's number
// of result slots; `launch(lane, reqs, n)` enqueues one launch of n requests
// (their slots already taken, slot_of set) on the lane's stream.
template <class Launch>
int pump_loop(fast_ctx *c, int nstreams, const std::vector<int> &nslots, const fast_pump_request *reqs, int nreq,
              int lanes, int limit, double max_seconds, double *done_s, int32_t *slot_of, int32_t *nbatches,
              Launch launch) {
    std::vector<std::vector<char>> busy(nstreams);
    for (int i = 0; i < nstreams; ++i) busy[i].assign(nslots[i], 0);
    int rc = FAST_OK;
    std::vector<PumpLane> lane(lanes);
    for (int k = 0; k < lanes; ++k) {
        PumpLane &L = lane[k];
        hipError_t e = hipSuccess;
        if (!c->pump_streams[k]) e = hipStreamCreateWithFlags(&c->pump_streams[k], hipStreamNonBlocking);
        L.stream = c->pump_streams[k];
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            rc = hip_fail(c, e, "pump lane setup");
            break;
        }
        L.reqs.reserve(limit);
    }
    std::vector<std::vector<int>> pending(nstreams);   // per stream, arrived requests in order
    std::vector<size_t> head(nstreams, 0);
    for (int r = 0; r < nreq; ++r) {
        done_s[r] = -1.0;
        slot_of[r] = -1;
    }
    int nb = 0, served = 0, next = 0;
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    // the oldest pending request of a stream with a free slot, or -1
    auto pick = [&]() {
        int best = -1;
        double when = 0.0;
        for (int i = 0; i < nstreams; ++i) {
            if (head[i] >= pending[i].size()) continue;
            if (std::find(busy[i].begin(), busy[i].end(), 0) == busy[i].end()) continue;
            const double a = reqs[pending[i][head[i]]].arrival_s;
            if (best < 0 || a < when) {
                best = i;
                when = a;
            }
        }
        return best;
    };
    while (rc == FAST_OK && served < nreq) {
        const double t = now();
        if (t > max_seconds) {
            rc = fail(c, FAST_ETIMEDOUT, "pump: max_seconds passed with requests unserved");
            break;
        }
        while (next < nreq && reqs[next].arrival_s <= t) {
            pending[reqs[next].stream].push_back(next);
            ++next;
        }
        for (PumpLane &L : lane) {   // completions
            if (!L.busy) continue;
            const hipError_t e = hipEventQuery(L.done);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) {
                rc = hip_fail(c, e, "pump launch");
                break;
            }
            const double tt = now();
            for (int r : L.reqs) {
                done_s[r] = tt;
                busy[reqs[r].stream][slot_of[r]] = 0;
            }
            served += (int)L.reqs.size();
            L.reqs.clear();
            L.busy = false;
        }
        for (PumpLane &L : lane) {   // launches
            if (rc != FAST_OK || L.busy) continue;
            while ((int)L.reqs.size() < limit) {
                const int i = pick();
                if (i < 0) break;
                const int r = pending[i][head[i]++];
                const int k = (int)(std::find(busy[i].begin(), busy[i].end(), 0) - busy[i].begin());
                busy[i][k] = 1;
                slot_of[r] = k;
                L.reqs.push_back(r);
            }
            if (L.reqs.empty()) break;
            rc = launch(L.stream, L.reqs.data(), (int)L.reqs.size());
            if (rc == FAST_OK) {
                const hipError_t e = hipEventRecord(L.done, L.stream);
                if (e != hipSuccess) rc = hip_fail(c, e, "pump event");
            }
            L.busy = true;   // drained below if anything failed
            ++nb;
        }
    }
    for (PumpLane &L : lane) {   // the streams stay with the context
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
    }
    *nbatches = nb;
    return rc;
}

int pump_args(fast_ctx *c, const fast_pump_stream *streams, int nstreams, const fast_pump_request *reqs, int nreq,
              int lanes, int max_batch, double max_seconds, const void *done_s, const void *nbatches) {
    if (!streams || !reqs || !done_s || !nbatches || nstreams < 1 || nreq < 1)
        return fail(c, FAST_EINVAL, "pump: NULL array, no stream or no request");
    if (lanes < 1 || lanes > FAST_PUMP_MAX_LANES) return fail(c, FAST_EINVAL, "pump: lanes not in 1..8");
    if (max_batch < 1 || max_batch > FAST_MAX_JOBS) return fail(c, FAST_EINVAL, "pump: max_batch out of range");
    if (!(max_seconds > 0.0)) return fail(c, FAST_EINVAL, "pump: max_seconds must be positive");
    return pump_check(c, streams, nstreams, reqs, nreq);
}

FG_API int fast_pump_run(fast_ctx *c, const fast_pump_stream *streams, int nstreams, const fast_pump_request *reqs,
                         int nreq, int lanes, int max_batch, int batched, double max_seconds, double *done_s,
                         int32_t *slot_of, int32_t *nbatches) {
    if (!c) return FAST_EINVAL;
    if (!slot_of) return fail(c, FAST_EINVAL, "pump: slot_of is NULL");
    int rc = pump_args(c, streams, nstreams, reqs, nreq, lanes, max_batch, max_seconds, done_s, nbatches);
    if (rc) return rc;
    for (int i = 0; i < nstreams; ++i) {
        const fast_pump_stream &S = streams[i];
        if (!S.out || (S.levels > 1 && !S.upper))
            return fail(c, FAST_EINVAL, "pump stream " + std::to_string(i) + " has no result slots");
        for (int k = 0; k < S.slots; ++k)
            if (!S.out[k] || (S.host_out && !S.host_out[k]))
                return fail(c, FAST_EINVAL, "pump stream " + std::to_string(i) + " has a NULL slot buffer");
    }
    DeviceGuard g(c->device);
    std::vector<int> nslots(nstreams);
    std::vector<size_t> out_bytes(nstreams);
    std::vector<std::vector<std::vector<fast_plane>>> planes(nstreams);   // per stream, slot: levels planes
    for (int i = 0; i < nstreams; ++i) {
        const fast_pump_stream &S = streams[i];
        int gw = 0, gh = 0;
        if (fast_grid_dims(S.pool[0].width, S.pool[0].height, S.cell, &gw, &gh) != FAST_OK)
            return fail(c, FAST_EINVAL, "pump stream " + std::to_string(i) + ": bad frame size or cell");
        out_bytes[i] = (size_t)gw * gh * sizeof(fast_feature);
        nslots[i] = S.slots;
        planes[i].resize(S.slots);
        for (int k = 0; k < S.slots; ++k) {
            planes[i][k].resize(S.levels);
            for (int l = 1; l < S.levels; ++l) planes[i][k][l] = S.upper[k * (S.levels - 1) + (l - 1)];
        }
    }
    std::vector<fast_job> jobs(batched ? max_batch : 1);
    auto launch = [&](hipStream_t s, const int *rq, int n) {
        for (int q = 0; q < n; ++q) {
            const fast_pump_request &R = reqs[rq[q]];
            const fast_pump_stream &S = streams[R.stream];
            std::vector<fast_plane> &pl = planes[R.stream][slot_of[rq[q]]];
            pl[0] = S.pool[R.frame % S.pool_frames];
            jobs[q] = fast_job{pl.data(), S.levels, S.t, S.n, S.cell, S.out[slot_of[rq[q]]], S.score};
        }
        int rc2;
        if (batched) {
            uint64_t tk = 0;
            rc2 = fast_submit(c, jobs.data(), n, s, &tk);
        } else {
            const fast_job &J = jobs[0];
            rc2 = fast_detect_grid_score(c, J.pyr, J.levels, J.t, J.n, J.cell, J.score, J.out, s);
        }
        for (int q = 0; rc2 == FAST_OK && q < n; ++q) {
            const fast_pump_request &R = reqs[rq[q]];
            const fast_pump_stream &S = streams[R.stream];
            if (!S.host_out) continue;
            const hipError_t e = hipMemcpyAsync(S.host_out[slot_of[rq[q]]], S.out[slot_of[rq[q]]], out_bytes[R.stream],
                                                hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) rc2 = hip_fail(c, e, "pump result copy");
        }
        return rc2;
    };
    return pump_loop(c, nstreams, nslots, reqs, nreq, lanes, batched ? max_batch : 1, max_seconds, done_s, slot_of,
                     nbatches, launch);
}

FG_API int fast_pump_run_frontend(fast_ctx *c, const fast_pump_stream *streams, const fast_pump_frontend *fe,
                                  int nstreams, const fast_pump_request *reqs, int nreq, int lanes, int max_batch,
                                  int mode, int max_iter, float eps, double max_seconds, double *done_s,
                                  int32_t *nbatches) {
    if (!c) return FAST_EINVAL;
    if (!fe) return fail(c, FAST_EINVAL, "pump: fe is NULL");
    int rc = pump_args(c, streams, nstreams, reqs, nreq, lanes, max_batch, max_seconds, done_s, nbatches);
    if (rc) return rc;
    rc = check_track_params(c, mode, max_iter, eps);
    if (rc) return rc;
    if (lanes > FAST_PUMP_MAX_LANES / 2) return fail(c, FAST_EINVAL, "pump: at most 4 front-end lanes");
    for (int i = 0; i < nstreams; ++i) {
        const fast_pump_frontend &F = fe[i];
        if (!F.grid || !F.feats || !F.count || !F.q || !F.status || !F.info || (streams[i].levels > 1 && !F.upper) ||
            F.capacity < 1 || F.capacity > FAST_MAX_TRACKS || F.redetect_below < 0 ||
            F.redetect_below > F.capacity)
            return fail(c, FAST_EINVAL, "pump front end " + std::to_string(i) + " is malformed");
    }
    DeviceGuard g(c->device);
    // per stream: the two alternating pyramids (level 0 set per frame), which
    // one is current, and whether a previous frame exists
    std::vector<std::array<std::vector<fast_plane>, 2>> pyr(nstreams);
    std::vector<int> cur(nstreams, 0), frames(nstreams, 0), nslots(nstreams, 1);
    for (int i = 0; i < nstreams; ++i) {
        const int L = streams[i].levels;
        for (int b = 0; b < 2; ++b) {
            pyr[i][b].resize(L);
            for (int l = 1; l < L; ++l) pyr[i][b][l] = fe[i].upper[b * (L - 1) + (l - 1)];
        }
    }
    std::vector<int32_t> slot_of(nreq);
    std::vector<fast_job> jobs(max_batch);
    std::vector<fast_frontend_job> fjobs(max_batch);
    auto launch = [&](hipStream_t s, const int *rq, int n) {
        for (int q = 0; q < n; ++q) {
            const fast_pump_request &R = reqs[rq[q]];
            const fast_pump_stream &S = streams[R.stream];
            std::vector<fast_plane> &pc = pyr[R.stream][cur[R.stream]];
            pc[0] = S.pool[R.frame % S.pool_frames];
            jobs[q] = fast_job{pc.data(), S.levels, S.t, S.n, S.cell, fe[R.stream].grid, FAST_SCORE_SADA};
        }
        uint64_t tk = 0;
        int rc2 = fast_submit(c, jobs.data(), n, s, &tk);
        if (rc2 != FAST_OK) return rc2;
        for (int q = 0; q < n; ++q) {
            const int i = reqs[rq[q]].stream;
            const fast_pump_frontend &F = fe[i];
            fjobs[q] = fast_frontend_job{frames[i] > 0 ? pyr[i][1 - cur[i]].data() : nullptr, pyr[i][cur[i]].data(),
                                         streams[i].levels, F.grid, streams[i].cell, F.capacity, F.redetect_below,
                                         F.feats, F.count, F.q, F.status, F.info};
        }
        rc2 = fast_frontend_step(c, fjobs.data(), n, mode, max_iter, eps, s, &tk);
        for (int q = 0; rc2 == FAST_OK && q < n; ++q) {
            const int i = reqs[rq[q]].stream;
            if (fe[i].info_host) {
                const hipError_t e = hipMemcpyAsync(fe[i].info_host, fe[i].info, 4 * sizeof(int32_t),
                                                    hipMemcpyDeviceToHost, s);
                if (e != hipSuccess) rc2 = hip_fail(c, e, "pump info copy");
            }
            cur[i] = 1 - cur[i];
            ++frames[i];
        }
        return rc2;
    };
    return pump_loop(c, nstreams, nslots, reqs, nreq, lanes, max_batch, max_seconds, done_s, slot_of.data(), nbatches,
                     launch);
}

FG_API int fast_poll(fast_ctx *c, uint64_t ticket) {
    if (!c) return FAST_EINVAL;
    DeviceGuard g(c->device);
    return ticket_state(c, ticket);
}

FG_API int fast_wait(fast_ctx *c, uint64_t ticket, int timeout_ms) {
    if (!c) return FAST_EINVAL;
    DeviceGuard g(c->device);
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        int st = ticket_state(c, ticket);
        if (st < 0) return st;
        if (st == 1) return FAST_OK;
        if (timeout_ms >= 0) {
            auto ms = std::chrono::duration_cast<std::chrono::milliseconds>(std::chrono::steady_clock::now() - t0);
            if (ms.count() >= timeout_ms) return fail(c, FAST_ETIMEDOUT, "wait timed out");
        }
        // poll without sleeping for the first 2 ms (a sleep costs tens of
        // microseconds of latency), then back off
        if (std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(2))
            std::this_thread::yield();
        else
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

FG_API int fast_plan_create(fast_ctx *c, const fast_job *jobs, int njobs, int flags, int *plan_id) {
    if (!c) return FAST_EINVAL;
    if (!plan_id) return fail(c, FAST_EINVAL, "plan_id is NULL");
    if (flags & ~FAST_PLAN_GRAPH) return fail(c, FAST_EINVAL, "unknown plan flags");
    std::vector<fg_job> table((size_t)(njobs > 0 ? njobs : 1));
    int total, total_upper, max_levels, mw1, mh1;
    bool all_single;
    int rc = build_table(c, jobs, njobs, table.data(), total, total_upper, max_levels, mw1, mh1, all_single);
    if (rc) return rc;
    DeviceGuard g(c->device);
    reap(c, false);   // a setup call: release what destroyed plans left behind
    Plan p;
    p.njobs = njobs;
    p.total = total;
    p.total_upper = total_upper;
    p.all_single = all_single;
    p.max_levels = max_levels;
    p.mw1 = mw1;
    p.mh1 = mh1;
    std::vector<fg_item> items((size_t)(total + total_upper));
    fill_items(table.data(), njobs, items.data());
    hipError_t e = hipMalloc((void **)&p.dev, sizeof(fg_job) * njobs);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc plan table");
    e = hipMalloc((void **)&p.items, sizeof(fg_item) * (total + total_upper));
    if (e != hipSuccess) { (void)hipFree(p.dev); return hip_fail(c, e, "hipMalloc plan item map"); }
    e = hipMalloc((void **)&p.counter, FG_COUNTER_WORDS * sizeof(unsigned));
    if (e != hipSuccess) {
        (void)hipFree(p.dev);
        (void)hipFree(p.items);
        return hip_fail(c, e, "hipMalloc plan counter");
    }
    e = hipMemcpy(p.dev, table.data(), sizeof(fg_job) * njobs, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p.items, items.data(), sizeof(fg_item) * (total + total_upper), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p.counter, 0, FG_COUNTER_WORDS * sizeof(unsigned));
    if (e == hipSuccess && (flags & FAST_PLAN_GRAPH)) {
        if (!c->capture_stream) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = fg_launch_batch(p.dev, p.items, njobs, total, total_upper, max_levels, mw1, mh1,
                                            all_single, p.counter,
                                            c->launch, c->capture_stream);
            e = hipStreamEndCapture(c->capture_stream, &p.graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        if (p.graph) (void)hipGraphDestroy(p.graph);
        (void)hipFree(p.dev);
        (void)hipFree(p.items);
        (void)hipFree(p.counter);
        return hip_fail(c, e, "plan creation");
    }
    p.live = true;
    c->plans.push_back(p);
    *plan_id = (int)c->plans.size() - 1;
    return FAST_OK;
}

FG_API int fast_plan_launch(fast_ctx *c, int plan_id, void *stream, uint64_t *ticket) {
    if (!c) return FAST_EINVAL;
    if (plan_id < 0 || plan_id >= (int)c->plans.size() || !c->plans[plan_id].live)
        return fail(c, FAST_EINVAL, "unknown plan");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    Plan &p = c->plans[plan_id];
    p.launched = true;
    p.last_stream = s;
    hipError_t e = p.exec ? hipGraphLaunch(p.exec, s)
                          : fg_launch_batch(p.dev, p.items, p.njobs, p.total, p.total_upper, p.max_levels, p.mw1, p.mh1,
                                            p.all_single,
                                            p.counter, c->launch, s);
    if (e != hipSuccess) return hip_fail(c, e, p.exec ? "hipGraphLaunch" : "plan launch");
    if (!ticket) return FAST_OK;
    return record_ticket(c, s, ticket);
}

FG_API int fast_plan_destroy(fast_ctx *c, int plan_id) {
    if (!c) return FAST_EINVAL;
    if (plan_id < 0 || plan_id >= (int)c->plans.size() || !c->plans[plan_id].live)
        return fail(c, FAST_EINVAL, "unknown plan");
    DeviceGuard g(c->device);
    Plan &p = c->plans[plan_id];
    // no host wait: the plan's memory and graph are released once the
    // launches already enqueued (all on p.last_stream) have completed
    Retired r;
    r.dev[0] = p.dev;
    r.dev[1] = p.items;
    r.dev[2] = p.counter;
    r.graph = p.graph;
    r.exec = p.exec;
    const int rc = retire(c, r, p.launched, p.last_stream);
    p = Plan();
    return rc;
}
