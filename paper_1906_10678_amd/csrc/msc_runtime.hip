// Host runtime and C ABI of libmsc: argument checks, the device workspace arena, the
// stage schedule of the reach search and the path search.  All arithmetic of the
// method runs in the kernels of msc_kernels.hip; this file plans memory, launches
// and copies results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "msc.h"
#include "msc_common.h"

using namespace msc;

struct ServerState;

// Device staging of msc_refine_static: a fixed buffer in the library's code object, so
// that call needs no device allocation.  Each device holds its own copy until the
// process ends; the host looks its address up once per device (static_scratch_init,
// from msc_ctx_create) and uses only that address, never the symbol itself.
static __device__ __align__(256) unsigned char scratch[MSC_REFINE_STATIC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: look up this device's copy of the buffer (once per device).
hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (char*)ptr;
    return hipSuccess;
}

char* static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

constexpr uint64_t kAlign = 256;
constexpr size_t kStagingBytes = 1 << 20;
constexpr int kCounters = 512;
constexpr int kMaxTickGrids = 64;   // grids of ticks per scene

struct TableEntry {
    short4* off;
    short4* sweep;
    unsigned int maxn2;
};

struct StageSet {
    SetView view{};
    uint64_t* list = nullptr;
    uint64_t count = 0;
    bool listed = false;
    bool used = false;
    bool at_top = false;   // dense, in the lane window's top stack (cleared after its last use)
    bool counted = true;   // false: built without a member count (count is meaningless)
};

}  // namespace

// One execution lane: a stream, a window of the workspace, pinned staging, counters
// and the bookkeeping of the call running on it.  The context's API calls use the
// control lane; batches and the server run one query at a time on each worker lane.
struct Lane {
    msc_ctx* owner = nullptr;
    int index = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* ws = nullptr;       // this lane's window of the workspace
    uint64_t lo = 0;          // per-call region grows up from 0
    uint64_t hi = 0;          // window size
    // Dense stage sets of a reach search are stacked down from the window's top and take
    // [hi - top, hi).  Below them, [clean, hi - top) is known to hold zeros once the work
    // queued so far has run.  The stacked sets are cleared after their last use, so the
    // next search's sets need no fill where they land in that region.
    uint64_t top = 0;
    uint64_t clean = 0;
    std::string err;
    unsigned long long* counters = nullptr;  // device
    int next_counter = 0;
    unsigned long long* ovf = nullptr;       // overflow counter of the current call
    char* staging = nullptr;                 // pinned, mapped host memory
    char* staging_dev = nullptr;             // its device address
    size_t staging_used = 0;
    unsigned long long publish_seq = 0;      // last sequence number given to k_publish
    msc_stats stats{};
    std::map<std::pair<int, int>, std::vector<uint64_t>> captured;
    int captured_n = 0;
    // MSC_PROFILE: one event pair per launch of the current call
    bool profiling = false;
    std::vector<hipEvent_t> events;
    std::vector<msc_timing> recs;
    int last_rec = -1;
};

struct msc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;  // the caller's stream (control lane)
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    uint64_t table_lo = 0;         // tables grow down from ws_bytes to table_lo
    uint64_t table_top = 0;
    std::mutex table_mu;
    std::map<std::tuple<int, int, int>, TableEntry> tables;
    Lane* control = nullptr;
    std::vector<Lane*> workers;
    std::string err;
    ServerState* server = nullptr;
    // launch shapes chosen by msc_autotune: variant per (kernel, log2 of the input
    // states); -1 = the default shape.  tune_force >= 0 makes every tunable launch use
    // that variant (while the tuner measures it).
    int8_t tune[MSC_K_COUNT][64];
    int tune_force = -1;
    msc_ctx() { std::memset(tune, -1, sizeof tune); }
};

// Grids of ticks of a scene with moving obstacles.  Slot 0 holds the static obstacles;
// slots 1.. hold the grids of recent ticks, each with the number of queries solving on
// it and an event recorded after it was written.  A slot is rewritten only when no
// query uses it.
struct GridSlot {
    uint64_t* grid = nullptr;
    int64_t tick = 0;
    int refs = 0;
    hipEvent_t ready = nullptr;
};
struct SceneDyn {
    std::mutex mu;
    std::vector<GridSlot> slot;
    int cur = 0;
};

// The solver reads only ctx .. bytes; a shallow copy with another grid and tick is how
// a query is solved on the grid of its tick.
struct msc_scene {
    msc_ctx* ctx = nullptr;
    int64_t tick = 0;
    int n = 0, wpr = 0, dilate = 0;
    uint64_t* grid = nullptr;   // the grid of the current tick
    uint64_t bytes = 0;
    SceneDyn* dyn = nullptr;    // null when the buffer holds only the static grid
    // recorded after the static grid's raster on the control lane's stream (which is
    // ordered after it); other lanes wait for it before their first use of the scene
    hipEvent_t ready = nullptr;
};

namespace {

msc_status fail(Lane* c, msc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        // the control lane's message is now the context's latest: drop an older one
        // left by a context-level call (msc_last_error prefers that one)
        if (c->owner && c == c->owner->control) c->owner->err.clear();
    }
    return st;
}

// Return any status other than MSC_OK (errors and "no answer" results alike).
#define MSC_TRY_STATUS(expr)             \
    do {                                 \
        msc_status s_ = (expr);          \
        if (s_ != MSC_OK) return s_;     \
    } while (0)

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(c, MSC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define MSC_TRY(expr)                       \
    do {                                    \
        msc_status s_ = (expr);             \
        if (s_ != MSC_OK) return s_;        \
    } while (0)

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Launch timing (MSC_PROFILE).
// The set expansions are timed by events carried on their own dispatch; other launches
// by events recorded on the stream around them.
bool timed_on_dispatch(int kernel) { return kernel == MSC_K_EXPAND_FWD || kernel == MSC_K_EXPAND_BWD; }

int prof_begin(Lane* c, int kernel, int stage, int64_t in) {
    c->last_rec = -1;
    (void)take_launch_events_used();
    if (!c->profiling) return -1;
    size_t idx = c->recs.size();
    while (c->events.size() < 2 * (idx + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        c->events.push_back(e);
    }
    if (timed_on_dispatch(kernel))
        set_launch_events(c->events[2 * idx], c->events[2 * idx + 1]);
    else if (hipEventRecord(c->events[2 * idx], c->stream) != hipSuccess)
        return -1;
    msc_timing t{};
    t.kernel = kernel;
    t.stage = stage;
    t.in_count = in;
    t.out_count = 0;
    t.ms = -1.0f;
    t.out_words = -1;
    c->recs.push_back(t);
    c->last_rec = (int)idx;
    return (int)idx;
}

void prof_end(Lane* c, int idx) {
    if (idx < 0) return;
    if (timed_on_dispatch(c->recs[idx].kernel)) {
        if (take_launch_events_used()) return;
        (void)hipEventRecord(c->events[2 * idx], c->stream);   // nothing was launched
    }
    (void)hipEventRecord(c->events[2 * idx + 1], c->stream);
}

void prof_out(Lane* c, int idx, int64_t out) {
    if (idx >= 0 && idx < (int)c->recs.size()) c->recs[idx].out_count = out;
}

void prof_words(Lane* c, int idx, int64_t words) {
    if (idx >= 0 && idx < (int)c->recs.size()) c->recs[idx].out_words = words;
}

void prof_finish(Lane* c) {
    if (!c->profiling) return;
    (void)hipStreamSynchronize(c->stream);
    for (size_t i = 0; i < c->recs.size(); ++i) {
        float ms = -1.0f;
        if (hipEventElapsedTime(&ms, c->events[2 * i], c->events[2 * i + 1]) == hipSuccess) c->recs[i].ms = ms;
    }
}

void prof_reset(Lane* c, uint32_t flags) {
    c->profiling = (flags & MSC_PROFILE) != 0;
    c->recs.clear();
    c->last_rec = -1;
}

#define LAUNCH(kind, stage, in, expr)                       \
    do {                                                    \
        int pi_ = prof_begin(c, (kind), (stage), (in));     \
        HIP_TRY(expr);                                      \
        prof_end(c, pi_);                                   \
    } while (0)

// Launch-shape variants the autotuner chooses from (variant 0 is the default).
constexpr Shape kShapes[] = {{16384, 0}, {4096, 0}, {65536, 0}, {16384, -1}, {16384, 1}, {1024, 0},
                             {512, 0},   {2048, 0}, {1024, -1}, {1024, 1}};
constexpr int kNumShapes = (int)(sizeof kShapes / sizeof kShapes[0]);

bool tunable(int kernel) {
    return kernel == MSC_K_EXPAND_FWD || kernel == MSC_K_EXPAND_BWD || kernel == MSC_K_JOIN || kernel == MSC_K_DMARK;
}

int size_class(uint64_t count) {
    int b = 0;
    while (b < 63 && (count >> (b + 1))) ++b;
    return b;
}

Shape shape_for(Lane* c, int kernel, uint64_t count) {
    const msc_ctx* o = c->owner;
    if (o->tune_force >= 0) return kShapes[o->tune_force];
    const int v = o->tune[kernel][size_class(count)];
    return v >= 0 && v < kNumShapes ? kShapes[v] : kShapes[0];
}

msc_status arena_alloc(Lane* c, uint64_t bytes, void** out) {
    uint64_t b = align_up(bytes ? bytes : 1);
    if (c->lo + b > c->hi - c->top) {
        return fail(c, MSC_E_NOMEM, "workspace exhausted: need %llu more bytes (used %llu of %llu)",
                    (unsigned long long)b, (unsigned long long)(c->lo + c->top), (unsigned long long)c->hi);
    }
    *out = c->ws + c->lo;
    c->lo += b;
    if (c->lo > c->clean) c->clean = c->lo;   // what this region held may be overwritten
    return MSC_OK;
}

uint64_t free_bytes(const Lane* c) { return c->hi - c->top > c->lo ? c->hi - c->top - c->lo : 0; }

// Shared table region at the top of the workspace (caller holds owner->table_mu).
msc_status persist_alloc(Lane* c, uint64_t bytes, void** out) {
    msc_ctx* o = c->owner;
    uint64_t b = align_up(bytes ? bytes : 1);
    if (o->table_top < b || o->table_top - b < o->table_lo) return fail(c, MSC_E_NOMEM, "table region exhausted");
    o->table_top -= b;
    *out = o->ws + o->table_top;
    return MSC_OK;
}

void begin_call(Lane* c) {
    c->lo = 0;
    if (c->top) c->clean = c->hi;   // sets left in the top stack by a failed call: nothing known
    c->top = 0;
    c->staging_used = 0;
    c->next_counter = 0;
    c->err.clear();
}

// A region of the pinned, device-mapped staging buffer: kernels read inputs from it
// and write small results into it directly (no copy); valid until the call ends.
msc_status host_area(Lane* c, size_t bytes, void** host, void** dev) {
    size_t b = (bytes + 255) & ~(size_t)255;
    if (c->staging_used + b > kStagingBytes - 4096) return fail(c, MSC_E_NOMEM, "staging buffer exhausted");
    *host = c->staging + c->staging_used;
    *dev = c->staging_dev + c->staging_used;
    c->staging_used += b;
    return MSC_OK;
}

// Upload a small host array through the pinned staging buffer (no host sync).
msc_status upload(Lane* c, const void* src, size_t bytes, void** dev) {
    void *h, *hd;
    MSC_TRY(host_area(c, bytes, &h, &hd));
    std::memcpy(h, src, bytes);
    MSC_TRY(arena_alloc(c, bytes, dev));
    HIP_TRY(hipMemcpyAsync(*dev, h, bytes, hipMemcpyHostToDevice, c->stream));
    return MSC_OK;
}

unsigned long long* take_counter(Lane* c) {
    if (c->next_counter >= kCounters) return nullptr;
    return c->counters + c->next_counter++;
}

// Stage sizes for the host: the publish kernel copies counters into mapped host memory
// and then bumps a sequence flag, which is polled (a few microseconds after the stage
// ends) instead of a stream synchronisation; after ~5 ms of polling the stream is
// synchronised, which also reports a failed launch.
// n <= 6 counters land at staging[end - 64 ..], the flag at staging[end - 8]
msc_status publish_and_wait(Lane* c, unsigned long long* dev, int n) {
    unsigned long long* hd = (unsigned long long*)(c->staging_dev + kStagingBytes - 64);
    volatile unsigned long long* hflag = (volatile unsigned long long*)(c->staging + kStagingBytes - 8);
    unsigned long long* dflag = (unsigned long long*)(c->staging_dev + kStagingBytes - 8);
    const unsigned long long seq = ++c->publish_seq;
    HIP_TRY(launch_publish(dev, hd, n, dflag, seq, c->stream));
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned spins = 0; *hflag != seq; ++spins) {
        if ((spins & 255) == 255 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(5)) {
            HIP_TRY(hipStreamSynchronize(c->stream));
            if (*hflag != seq) return fail(c, MSC_E_HIP, "stage counter was not published");
            break;
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return MSC_OK;
}

msc_status read_counter(Lane* c, unsigned long long* dev, uint64_t* out) {
    MSC_TRY(publish_and_wait(c, dev, 1));
    *out = *(volatile unsigned long long*)(c->staging + kStagingBytes - 64);
    return MSC_OK;
}

// Waits until everything queued on the lane's stream so far has run (results that
// kernels wrote to mapped host memory are then visible).
msc_status sync_lane(Lane* c) { return publish_and_wait(c, nullptr, 0); }

int64_t isqrt_ceil(int64_t v) {
    int64_t r = 0;
    while (r * r < v) {
        int64_t step = 1;
        while ((r + step * 2) * (r + step * 2) < v) step *= 2;
        r += step;
    }
    return r;
}

uint64_t pow2_at_least(uint64_t v) {
    uint64_t p = 64;
    while (p < v) p <<= 1;
    return p;
}

// ---------------------------------------------------------------------------
// Arm plan: the arm in steps, joint windows, reference angles.
// ---------------------------------------------------------------------------
struct Plan {
    int n, na, S;
    int base[3];
    int ia0, ie0;
    int type[kMaxDof], len[kMaxDof], lo[kMaxDof], hi[kMaxDof], ref[kMaxDof];
    int target[3];
    int prune;
    int count_sets;   // MSC_COUNT_SETS: member counts and output words of every stage
    int split;   // -1 adaptive
    int app_az, app_el, app_half;   // approach cone of the last segment (centidegrees; half < 0: none)
};

msc_status set_approach(Lane* c, const msc_opts& o, Plan& p) {
    if (o.approach_half_cdeg > 18000) return fail(c, MSC_E_ARG, "approach half-angle above 18000 cdeg");
    p.app_az = o.approach_az_cdeg;
    p.app_el = o.approach_el_cdeg;
    p.app_half = o.approach_half_cdeg < 0 ? -1 : o.approach_half_cdeg;
    return MSC_OK;
}

// Final orientations inside the approach cone, as rows of na bits per azimuth index
// (word ia * 4 + ie / 64, bit ie % 64): d(ia, ie) . a >= cos(half) - 1e-9 in FP64.
void approach_rows(const Plan& p, uint64_t* rows) {
    constexpr double kPi = 3.14159265358979323846;
    const double deg = kPi / 180.0;
    const double az = p.app_az / 100.0 * deg, el = p.app_el / 100.0 * deg;
    const double ax = std::cos(el) * std::cos(az), ay = std::cos(el) * std::sin(az), azz = std::sin(el);
    const double lim = std::cos(p.app_half / 100.0 * deg) - 1e-9;
    const double step = 360.0 / p.na;
    std::memset(rows, 0, sizeof(uint64_t) * 4 * (size_t)p.na);
    for (int ia = 0; ia < p.na; ++ia) {
        const double a = ia * step * deg;
        for (int ie = 0; ie < p.na; ++ie) {
            const double e = ie * step * deg;
            const double dot = std::cos(e) * std::cos(a) * ax + std::cos(e) * std::sin(a) * ay + std::sin(e) * azz;
            if (dot >= lim) rows[(size_t)ia * 4 + (ie >> 6)] |= 1ull << (ie & 63);
        }
    }
}

msc_status check_arm(Lane* c, const msc_arm* arm, int grid_n) {
    if (!arm) return fail(c, MSC_E_ARG, "arm is NULL");
    if (arm->dof < 1 || arm->dof > MSC_MAX_DOF) return fail(c, MSC_E_ARG, "dof %d outside 1..%d", arm->dof, MSC_MAX_DOF);
    if (arm->step_cdeg <= 0 || 36000 % arm->step_cdeg) return fail(c, MSC_E_ARG, "step_cdeg must divide 36000");
    int na = 36000 / arm->step_cdeg;
    if (na > kMaxNa) return fail(c, MSC_E_ARG, "more than %d orientation bins", kMaxNa);
    if (arm->samples < 1 || arm->samples > 64) return fail(c, MSC_E_ARG, "samples outside 1..64");
    if (arm->az0_cdeg % arm->step_cdeg || arm->el0_cdeg % arm->step_cdeg)
        return fail(c, MSC_E_ARG, "initial orientation not a multiple of the step");
    for (int k = 0; k < arm->dof; ++k) {
        if (arm->type[k] != MSC_YAW && arm->type[k] != MSC_PITCH) return fail(c, MSC_E_ARG, "joint %d type", k);
        if (arm->len_vox[k] < 0 || arm->len_vox[k] > 4096) return fail(c, MSC_E_ARG, "joint %d length", k);
        if (arm->lo_cdeg[k] % arm->step_cdeg || arm->hi_cdeg[k] % arm->step_cdeg)
            return fail(c, MSC_E_ARG, "joint %d limits not multiples of the step", k);
        if (arm->lo_cdeg[k] > arm->hi_cdeg[k]) return fail(c, MSC_E_ARG, "joint %d lo > hi", k);
        if (arm->lo_cdeg[k] < -36000 || arm->hi_cdeg[k] > 36000)
            return fail(c, MSC_E_ARG, "joint %d limits beyond one turn", k);
        int L = (arm->hi_cdeg[k] - arm->lo_cdeg[k]) / arm->step_cdeg + 1;
        if (L > kMaxNa) return fail(c, MSC_E_ARG, "joint %d has more than %d angles", k, kMaxNa);
    }
    for (int i = 0; i < 3; ++i)
        if (arm->base[i] < 0 || arm->base[i] >= grid_n) return fail(c, MSC_E_ARG, "base outside the grid");
    return MSC_OK;
}

void make_plan(const msc_arm* arm, const int32_t* target, Plan& p) {
    p.n = arm->dof;
    p.na = 36000 / arm->step_cdeg;
    p.S = arm->samples;
    for (int i = 0; i < 3; ++i) p.base[i] = arm->base[i];
    auto wrap = [&](int v) { return ((v % p.na) + p.na) % p.na; };
    p.ia0 = wrap(arm->az0_cdeg / arm->step_cdeg);
    p.ie0 = wrap(arm->el0_cdeg / arm->step_cdeg);
    for (int k = 0; k < p.n; ++k) {
        p.type[k] = arm->type[k];
        p.len[k] = arm->len_vox[k];
        p.lo[k] = arm->lo_cdeg[k] / arm->step_cdeg;
        p.hi[k] = arm->hi_cdeg[k] / arm->step_cdeg;
        p.ref[k] = 0;
    }
    for (int i = 0; i < 3; ++i) p.target[i] = target ? target[i] : 0;
    p.prune = 1;
    p.count_sets = 0;
    p.split = -1;
    p.app_az = p.app_el = 0;
    p.app_half = -1;
}

msc_status get_table(Lane* c, int na, int S, int L, TableEntry* out) {
    // tables are shared by all lanes: built once per (na, S, L) under the owner's lock
    std::lock_guard<std::mutex> lock(c->owner->table_mu);
    auto& tables = c->owner->tables;
    auto key = std::make_tuple(na, S, L);
    auto it = tables.find(key);
    if (it != tables.end()) {
        *out = it->second;
        return MSC_OK;
    }
    TableEntry t{};
    void* p;
    MSC_TRY(persist_alloc(c, (uint64_t)na * na * sizeof(short4), &p));
    t.off = (short4*)p;
    MSC_TRY(persist_alloc(c, (uint64_t)na * na * S * sizeof(short4), &p));
    t.sweep = (short4*)p;
    unsigned int* d_max;
    MSC_TRY(persist_alloc(c, 256, &p));
    d_max = (unsigned int*)p;
    HIP_TRY(launch_fill((uint64_t*)d_max, 1, 0ull, c->stream));
    HIP_TRY(launch_tables(na, S, L, t.off, t.sweep, d_max, c->stream));
    unsigned int* h = (unsigned int*)(c->staging + kStagingBytes - 128);
    HIP_TRY(hipMemcpyAsync(h, d_max, sizeof(unsigned int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    t.maxn2 = *h;
    tables[key] = t;
    *out = t;
    return MSC_OK;
}

GridView grid_view(const msc_scene* s) { return GridView{s->grid, s->n, s->wpr}; }

// A query's hold on the grid of its scene's current tick.
struct Binding {
    SceneDyn* dyn = nullptr;
    int slot = -1;
    msc_scene view{};           // the scene with the bound grid and tick
    hipEvent_t ready = nullptr; // wait for it on a stream other than the one that wrote the grid
};

Binding bind_scene(const msc_scene* s) {
    Binding b;
    if (!s) return b;
    if (!s->dyn) {
        b.view = *s;
    } else {
        // msc_scene_set_dynamic changes grid and tick under the same lock
        std::lock_guard<std::mutex> lock(s->dyn->mu);
        b.view = *s;
        b.dyn = s->dyn;
        b.slot = s->dyn->cur;
        GridSlot& g = s->dyn->slot[b.slot];
        ++g.refs;
        b.view.grid = g.grid;
        b.view.tick = g.tick;
        b.ready = g.ready;
    }
    return b;
}

void unbind_scene(Binding& b) {
    if (b.dyn && b.slot >= 0) {
        std::lock_guard<std::mutex> lock(b.dyn->mu);
        --b.dyn->slot[b.slot].refs;
    }
    b.dyn = nullptr;
    b.slot = -1;
}

// Voxel box of the states after k segments: within sum_{j<=k} R_j of the base and
// sum_{j>k} R_j of the target (the pruning radii), clipped to the grid.
struct Box {
    int x0, y0, z0, nx, ny, nz;
    bool empty() const { return nx <= 0 || ny <= 0 || nz <= 0; }
    uint64_t voxels() const { return empty() ? 0 : (uint64_t)nx * ny * nz; }
};

Box stage_box(const Plan& p, int N, const std::vector<int64_t>& R, int k) {
    int64_t rb = 0, rt = 0;
    for (int j = 0; j < k; ++j) rb += R[j];
    for (int j = k; j < p.n; ++j) rt += R[j];
    Box b;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        int64_t l = 0, h = N - 1;
        if (p.prune) {
            l = std::max<int64_t>(l, std::max<int64_t>(p.base[a] - rb, p.target[a] - rt));
            h = std::min<int64_t>(h, std::min<int64_t>(p.base[a] + rb, p.target[a] + rt));
        }
        lo[a] = (int)l;
        hi[a] = (int)h;
    }
    b.x0 = lo[0];
    b.y0 = lo[1];
    b.z0 = lo[2];
    b.nx = hi[0] - lo[0] + 1;
    b.ny = hi[1] - lo[1] + 1;
    b.nz = hi[2] - lo[2] + 1;
    return b;
}

// Allocate and clear the structure of one stage set: a dense bitset over the stage box
// when it is no larger than a hash table sized for `upper` states, else the hash table.
// A dense set pushed onto the lane window's top stack: only the part of it not known to
// hold zeros is filled.
msc_status top_alloc(Lane* c, uint64_t words, uint64_t** out) {
    const uint64_t b = align_up(words * 8);
    const uint64_t end = c->hi - c->top;   // the stack's current bottom
    if (b > end || end - b < c->lo)
        return fail(c, MSC_E_NOMEM, "workspace exhausted: need %llu more bytes", (unsigned long long)b);
    const uint64_t base = end - b;
    const uint64_t known = std::min(std::max(c->clean, base), end);   // [known, end) holds zeros
    if (base < known)
        LAUNCH(MSC_K_FILL, -1, (int64_t)((known - base) / 8),
               launch_fill((uint64_t*)(c->ws + base), (known - base) / 8, 0ull, c->stream));
    c->top += b;
    *out = (uint64_t*)(c->ws + base);
    return MSC_OK;
}

msc_status make_set(Lane* c, const Plan& p, const Box& box, uint64_t upper, int fast_ia, bool force_dense,
                    StageSet& s, bool at_top = false) {
    const uint64_t na2 = (uint64_t)p.na * p.na;
    uint64_t dense_words = box.empty() ? 0 : (box.voxels() * na2 + 63) / 64 + 1;
    uint64_t hash_slots = pow2_at_least(std::max<uint64_t>(2 * upper, 64));
    // Dense sets take a run of predecessors in 1-3 atomicOr and a membership test in one
    // load, where a hash set needs a CAS chain per state: dense is preferred up to 8x the
    // hash table's bytes, as long as it leaves half of the lane's free workspace.
    const uint64_t room = free_bytes(c);
    bool dense = !box.empty() &&
                 (force_dense || (dense_words <= 8 * hash_slots && dense_words * 8 <= room / 2) ||
                  dense_words <= hash_slots);
    s = StageSet();
    s.view.na = p.na;
    s.used = true;
    void* mem;
    if (dense) {
        s.view.kind = kDense;
        s.view.fast_ia = fast_ia;
        s.view.x0 = box.x0;
        s.view.y0 = box.y0;
        s.view.z0 = box.z0;
        s.view.nx = box.nx;
        s.view.ny = box.ny;
        s.view.nz = box.nz;
        s.view.cap = dense_words;
        if (at_top) {
            MSC_TRY(top_alloc(c, dense_words, &s.view.words));
            s.at_top = true;
        } else {
            MSC_TRY(arena_alloc(c, dense_words * 8, &mem));
            s.view.words = (uint64_t*)mem;
            LAUNCH(MSC_K_FILL, -1, (int64_t)dense_words, launch_fill(s.view.words, dense_words, 0ull, c->stream));
        }
    } else {
        s.view.kind = kHash;
        s.view.cap = hash_slots;
        MSC_TRY(arena_alloc(c, hash_slots * 8, &mem));
        s.view.words = (uint64_t*)mem;
        LAUNCH(MSC_K_FILL, -2, (int64_t)hash_slots, launch_fill(s.view.words, hash_slots, kEmpty, c->stream));
    }
    return MSC_OK;
}

msc_status ensure_list(Lane* c, StageSet& s) {
    if (s.listed) return MSC_OK;
    void* mem;
    MSC_TRY(arena_alloc(c, std::max<uint64_t>(s.count, 1) * 8, &mem));
    s.list = (uint64_t*)mem;
    unsigned long long* ctr = take_counter(c);
    if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
    LAUNCH(MSC_K_COMPACT, -1, (int64_t)s.count, launch_compact(s.view, s.list, s.count, ctr, c->ovf, c->stream));
    s.listed = true;
    return MSC_OK;
}

// Copy a set's members to the host as sorted keys ((z*N + y)*N + x) << 16 | ia << 8 | ie.
msc_status capture_set(Lane* c, StageSet& s, int N, int which, int stage) {
    std::vector<uint64_t> keys;
    if (s.count) {
        void* mem;
        MSC_TRY(arena_alloc(c, s.count * 8, &mem));
        uint64_t* lst = (uint64_t*)mem;
        unsigned long long* ctr = take_counter(c);
        if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
        HIP_TRY(launch_compact(s.view, lst, s.count, ctr, c->ovf, c->stream));
        uint64_t got = 0;
        MSC_TRY(read_counter(c, ctr, &got));
        keys.resize(std::min<uint64_t>(got, s.count));
        HIP_TRY(hipMemcpyAsync(keys.data(), lst, keys.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    for (auto& k : keys) {
        int x, y, z, ia, ie;
        unpack_key(k, x, y, z, ia, ie);
        k = ((((uint64_t)z * N + y) * N + x) << 16) | ((uint64_t)ia << 8) | (uint64_t)ie;
    }
    std::sort(keys.begin(), keys.end());
    c->captured[{which, stage}] = std::move(keys);
    return MSC_OK;
}

struct ReachOut {
    std::vector<int32_t> sols;  // nsol * n
    int nsol = 0;
};

msc_status check_overflow(Lane* c, unsigned long long* ovf, const char* what) {
    uint64_t v = 0;
    MSC_TRY(read_counter(c, ovf, &v));
    if (v) return fail(c, MSC_E_CAPACITY, "%s overflowed (%llu states without room)", what, (unsigned long long)v);
    return MSC_OK;
}

// Measurement (MSC_COUNT_SETS): the non-zero words of a set's structure, stored in
// launch record rec (the count runs after the timed launch).
msc_status count_words(Lane* c, const SetView& v, int rec) {
    unsigned long long* ctr = take_counter(c);
    if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
    HIP_TRY(launch_count_words(v, ctr, c->stream));
    uint64_t words = 0;
    MSC_TRY(read_counter(c, ctr, &words));
    prof_words(c, rec, (int64_t)words);
    return MSC_OK;
}

// The staged reach search.  Returns MSC_OK with up to `want` solutions (steps) in the
// canonical order, or MSC_NO_REACH.
msc_status run_reach(Lane* c, const msc_scene* sc, const Plan& p, int want, bool capture, ReachOut& out) {
    const int n = p.n, na = p.na, N = sc->n;
    const GridView g = grid_view(sc);
    std::memset(&c->stats, 0, sizeof c->stats);
    c->stats.dof = n;
    c->captured.clear();
    c->captured_n = N;
    out = ReachOut();

    LAUNCH(MSC_K_FILL, -1, 0, launch_fill((uint64_t*)c->counters, kCounters, 0ull, c->stream));
    c->ovf = take_counter(c);

    // Tables and pruning radii R_j = ceil(max_o |off_j[o]|).
    std::vector<JointView> jv(n);
    std::vector<int64_t> R(n);
    for (int k = 0; k < n; ++k) {
        TableEntry t;
        MSC_TRY(get_table(c, na, p.S, p.len[k], &t));
        jv[k] = JointView{t.off, t.sweep, p.type[k], p.lo[k], p.hi[k], p.S};
        R[k] = isqrt_ceil((int64_t)t.maxn2);
    }
    // Orientation reachability rows O_k (k = 0..n).
    uint64_t *rows_ie = nullptr, *rows_ia = nullptr;
    {
        void *m1, *m2;
        MSC_TRY(arena_alloc(c, (uint64_t)(n + 1) * na * 4 * 8, &m1));
        MSC_TRY(arena_alloc(c, (uint64_t)(n + 1) * na * 4 * 8, &m2));
        rows_ie = (uint64_t*)m1;
        rows_ia = (uint64_t*)m2;
        OrientArgs oa{};
        oa.n = n;
        oa.na = na;
        oa.ia0 = p.ia0;
        oa.ie0 = p.ie0;
        for (int k = 0; k < n; ++k) {
            oa.type[k] = p.type[k];
            oa.lo[k] = p.lo[k];
            oa.hi[k] = p.hi[k];
        }
        LAUNCH(MSC_K_ORIENT, -1, 0, launch_orient(oa, rows_ie, rows_ia, c->stream));
    }
    auto rows_for = [&](int stage, int yaw) -> const uint64_t* {
        if (!p.prune) return nullptr;
        return (yaw ? rows_ia : rows_ie) + (size_t)stage * na * 4;
    };

    std::vector<StageSet> F(n + 1), B(n + 1);
    std::vector<Box> box(n + 1);
    for (int k = 0; k <= n; ++k) box[k] = stage_box(p, N, R, k);

    // Seeds: both sets with their lists, both counts in one host round trip.
    {
        Box b0{p.base[0], p.base[1], p.base[2], 1, 1, 1};
        MSC_TRY(make_set(c, p, b0, 1, 0, false, F[0]));
        Box bn{p.target[0], p.target[1], p.target[2], 1, 1, 1};
        int fast = p.type[n - 1] == MSC_YAW ? 1 : 0;
        MSC_TRY(make_set(c, p, bn, (uint64_t)na * na, fast, true, B[n]));
        void *l0, *ln;
        MSC_TRY(arena_alloc(c, 8, &l0));
        MSC_TRY(arena_alloc(c, (uint64_t)na * na * 8, &ln));
        unsigned long long* ctr = take_counter(c);
        unsigned long long* ctr2 = take_counter(c);
        if (!ctr || ctr2 != ctr + 1) return fail(c, MSC_E_CAPACITY, "out of counters");
        LAUNCH(MSC_K_SEED, 0, 0,
               launch_seed_fwd(F[0].view, g, p.base[0], p.base[1], p.base[2], p.ia0, p.ie0, (uint64_t*)l0, ctr,
                               c->stream));
        const uint64_t* cone = nullptr;
        if (p.app_half >= 0) {
            void *hc, *dc;
            MSC_TRY(host_area(c, sizeof(uint64_t) * 4 * (size_t)na, &hc, &dc));
            approach_rows(p, (uint64_t*)hc);
            cone = (const uint64_t*)dc;
        }
        LAUNCH(MSC_K_SEED, n, 0,
               launch_seed_bwd(B[n].view, g, p.target[0], p.target[1], p.target[2], rows_for(n, 0), p.prune, cone,
                               (uint64_t*)ln, ctr2, c->stream));
        MSC_TRY(publish_and_wait(c, ctr, 2));
        const volatile unsigned long long* h = (const volatile unsigned long long*)(c->staging + kStagingBytes - 64);
        F[0].count = h[0];
        B[n].count = h[1];
        F[0].list = (uint64_t*)l0;
        F[0].listed = true;
        B[n].list = (uint64_t*)ln;
        B[n].listed = true;
    }
    bool empty = F[0].count == 0 || B[n].count == 0;
    int kf = 0, kb = n;
    unsigned long long* ovf = c->ovf;
    // Forward stage k from F_{k-1}'s list into `out`.
    auto expand_forward = [&](int k, StageSet& out, bool top) -> msc_status {
        MSC_TRY(ensure_list(c, F[k - 1]));
        uint64_t upper = F[k - 1].count * (uint64_t)(p.hi[k - 1] - p.lo[k - 1] + 1);
        int fast = (k < n && p.type[k] == MSC_YAW) ? 1 : 0;
        MSC_TRY(make_set(c, p, box[k], upper, fast, false, out, top));
        int64_t rt = 0;
        for (int j = k; j < n; ++j) rt += R[j];
        long long r2 = p.prune ? (long long)(rt * rt) : -1;
        unsigned long long* ctr = take_counter(c);
        if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
        LAUNCH(MSC_K_EXPAND_FWD, k, (int64_t)F[k - 1].count,
               launch_expand_fwd(F[k - 1].list, F[k - 1].count, out.view, g, jv[k - 1], p.target[0], p.target[1],
                                 p.target[2], r2, ctr, ovf, c->stream, shape_for(c, MSC_K_EXPAND_FWD, F[k - 1].count)));
        const int rec = c->last_rec;
        MSC_TRY(read_counter(c, ctr, &out.count));
        prof_out(c, rec, (int64_t)out.count);
        if (p.count_sets && rec >= 0) MSC_TRY(count_words(c, out.view, rec));
        return MSC_OK;
    };
    // The two pathways are expanded until they are one transition apart, then met
    // (split 0: the backward pathway runs down to the root and is joined with F_0).
    auto finished = [&]() { return p.split == 0 ? kb == 0 : kb - kf == 1; };
    auto window = [&](int k) { return (double)(p.hi[k] - p.lo[k] + 1); };
    // Rough per-item device times that steer the split (the result does not depend on
    // it): a forward candidate (state x angle), a backward input state (expansion plus
    // its list), a meet candidate against a small dense B (cache resident) or against
    // a large or hashed one, and fill bandwidth.
    constexpr double kFwdNs = 33.0, kBwdNs = 100.0, kMeetSmallNs = 4.0, kMeetBigNs = 12.0;
    constexpr double kFillBytesPerNs = 4500.0, kMallBytes = 256.0 * (1 << 20);
    auto meet_ns = [&](const StageSet& b) {
        return (b.view.kind == kDense && 8.0 * (double)b.view.cap <= kMallBytes) ? kMeetSmallNs : kMeetBigNs;
    };
    // Cost of one more backward stage from B_kb plus the meet from F_kf.
    auto backward_then_meet = [&](int kf_, int kb_) {
        const uint64_t upper = B[kb_].count * (uint64_t)window(kb_ - 1);
        const uint64_t dense_words = box[kb_ - 1].voxels() * (uint64_t)na * na / 64;
        const uint64_t slots = pow2_at_least(std::max<uint64_t>(2 * upper, 64));
        const uint64_t words = dense_words <= 8 * slots ? dense_words : slots;
        const bool dense = dense_words <= 8 * slots;
        const double meet = (dense && 8.0 * (double)dense_words <= kMallBytes) ? kMeetSmallNs : kMeetBigNs;
        return (double)B[kb_].count * kBwdNs + 8.0 * (double)words / kFillBytesPerNs +
               (double)F[kf_].count * window(kf_) * meet;
    };
    bool backward_only = false;
    while (!empty && !finished()) {
        bool forward;
        if (p.split >= 0) {
            forward = p.split >= 1 && kf < p.split - 1;
        } else if (backward_only) {
            forward = false;
        } else {
            const double cf = (double)F[kf].count * window(kf);
            const double cb = (double)B[kb].count * 3.0;
            forward = cf <= cb;
            if (kb - kf == 2 && kf >= 1 && F[kf - 1].count > 0) {
                // The last step before the meet decides which sets meet: estimate the next
                // forward set from the last growth (damped: growth slows as the pruning
                // ball shrinks) and compare the two ways to the meet.
                const double grow = 0.5 * (double)F[kf].count / (double)F[kf - 1].count;
                const double next = (double)F[kf].count * std::max(1.0, grow);
                const double fwd = cf * kFwdNs + next * window(kf + 1) * meet_ns(B[kb]);
                forward = fwd <= backward_then_meet(kf, kb);
            }
        }
        if (forward) {
            MSC_TRY(expand_forward(kf + 1, F[kf + 1], true));
            kf = kf + 1;
            empty = F[kf].count == 0;
            // The step before the meet, checked with the real size: when the meet from F_kf
            // is dearer than one more backward stage plus the meet from F_{kf-1}, the
            // forward side steps back (F_kf stays built but unused).
            if (!empty && p.split < 0 && kb - kf == 1 && kf >= 1) {
                const double meet_here = (double)F[kf].count * window(kf) * meet_ns(B[kb]);
                if (backward_then_meet(kf - 1, kb) < meet_here) {
                    kf -= 1;
                    backward_only = true;
                }
            }
        } else {
            const int k = kb;  // joint k-1 (0-based) lays segment k; produce B_{k-1}
            MSC_TRY(ensure_list(c, B[kb]));
            uint64_t upper = B[kb].count * (uint64_t)(p.hi[k - 1] - p.lo[k - 1] + 1);
            int yaw = p.type[k - 1] == MSC_YAW ? 1 : 0;
            // The set the meet probes needs no member count (an empty one simply meets
            // nothing): it is built without one, and without a host round trip, unless
            // the sets are captured.
            const bool last = p.split == 0 ? k - 1 == 0 : k - 1 - kf == 1;
            MSC_TRY(make_set(c, p, box[k - 1], upper, yaw, false, B[k - 1], true));
            int64_t rb = 0;
            for (int j = 0; j < k - 1; ++j) rb += R[j];
            long long r2 = p.prune ? (long long)(rb * rb) : -1;
            const bool count = capture || !last || p.count_sets;
            unsigned long long* ctr = count ? take_counter(c) : nullptr;
            if (count && !ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
            LAUNCH(MSC_K_EXPAND_BWD, k - 1, (int64_t)B[kb].count,
                   launch_expand_bwd(B[kb].list, B[kb].count, B[k - 1].view, g, jv[k - 1], p.base[0], p.base[1],
                                     p.base[2], r2, rows_for(k - 1, yaw), ctr, ovf, c->stream, shape_for(c, MSC_K_EXPAND_BWD, B[kb].count)));
            kb = k - 1;
            if (count) {
                const int rec = c->last_rec;
                MSC_TRY(read_counter(c, ctr, &B[k - 1].count));
                prof_out(c, rec, (int64_t)B[k - 1].count);
                if (p.count_sets && rec >= 0) MSC_TRY(count_words(c, B[k - 1].view, rec));
                empty = B[k - 1].count == 0;
            } else {
                B[k - 1].counted = false;
            }
        }
    }
    // Clears the stage sets in the window's top stack once nothing reads them any more
    // (after the canonical walk), so that the top of the window is clean again: a set
    // built by the backward stage from the words that stage can have written (its input
    // list), a forward set from its own list (the words of its members), each only when
    // that list is shorter than an eighth of the set's words (a state costs about as much
    // as a fill of 8 words), else by a fill.
    auto release_top = [&]() -> msc_status {
        for (int k = 0; k <= n; ++k) {
            StageSet* sets[2] = {&F[k], &B[k]};
            for (int side = 0; side < 2; ++side) {
                StageSet& st = *sets[side];
                if (!st.at_top) continue;
                const uint64_t cap = st.view.cap;
                const bool run_rows = side == 1 && k < n && B[k + 1].listed && B[k + 1].count < cap / 8 &&
                                      ((st.view.fast_ia != 0) == (jv[k].type == MSC_YAW));
                if (run_rows)
                    LAUNCH(MSC_K_FILL, k, (int64_t)B[k + 1].count,
                           launch_unexpand_bwd(B[k + 1].list, B[k + 1].count, st.view, jv[k], c->stream));
                else if (side == 0 && st.listed && st.count < cap / 8)
                    LAUNCH(MSC_K_FILL, k, (int64_t)st.count, launch_unlist(st.list, st.count, st.view, c->stream));
                else
                    LAUNCH(MSC_K_FILL, -1, (int64_t)cap, launch_fill(st.view.words, cap, 0ull, c->stream));
                st.at_top = false;
            }
        }
        c->clean = std::min(c->clean, c->hi - c->top);
        c->top = 0;
        return MSC_OK;
    };
    MSC_TRY(check_overflow(c, ovf, "a stage set"));
    const int m = kb;
    c->stats.split_m = m;
    for (int k = 0; k <= n; ++k) {
        c->stats.fwd_count[k] = F[k].used ? (int64_t)F[k].count : -1;
        c->stats.bwd_count[k] = !B[k].used ? -1 : B[k].counted ? (int64_t)B[k].count : -2;
        c->stats.fwd_dense[k] = F[k].used && F[k].view.kind == kDense;
        c->stats.bwd_dense[k] = B[k].used && B[k].view.kind == kDense;
    }
    if (capture) {
        for (int k = 0; k <= n; ++k) {
            if (F[k].used) MSC_TRY(capture_set(c, F[k], N, 0, k));
            if (B[k].used) MSC_TRY(capture_set(c, B[k], N, 1, k));
        }
    }
    if (empty) {
        MSC_TRY(release_top());
        return MSC_NO_REACH;
    }

    // C_m and the D sets.  Stage sets used by the canonical walk: D_k (k < m) in F_k's
    // structure, C_m (or B_m, equivalent for the walk) at stage m, B_k for k > m.
    StageSet Cset;
    uint64_t joined = 0;
    if (m == 0) {
        MSC_TRY(ensure_list(c, F[0]));
        unsigned long long* jc = take_counter(c);
        LAUNCH(MSC_K_JOIN, 0, (int64_t)F[0].count, launch_join(F[0].list, F[0].count, F[0].view, B[0].view, jc, c->stream));
        MSC_TRY(read_counter(c, jc, &joined));
        Cset = F[0];
    } else {
        if (capture) {
            // F_m itself is only built for the dump
            StageSet Fm;
            MSC_TRY(expand_forward(m, Fm, false));
            MSC_TRY(capture_set(c, Fm, N, 0, m));
        }
        MSC_TRY(ensure_list(c, F[m - 1]));
        const int fast = (m < n && p.type[m] == MSC_YAW) ? 1 : 0;
        int64_t rt_m = 0;
        for (int j = m; j < n; ++j) rt_m += R[j];
        const long long meet_r2 = p.prune ? (long long)(rt_m * rt_m) : -1;
        if (!capture) {
            // Only D_{m-1} is needed: the canonical walk steps from D_{m-1} into B_m,
            // which for a clear move is the same as stepping into C_m; C is not built.
            unsigned long long* hc = take_counter(c);
            unsigned long long* kc = take_counter(c);
            if (!hc || !kc) return fail(c, MSC_E_CAPACITY, "out of counters");
            LAUNCH(MSC_K_JOIN, m, (int64_t)F[m - 1].count,
                   launch_meet(F[m - 1].list, F[m - 1].count, F[m - 1].view, B[m].view, B[m].view, g, jv[m - 1],
                               kMeetMark, hc, kc, ovf, p.target[0], p.target[1], p.target[2], meet_r2, c->stream, shape_for(c, MSC_K_JOIN, F[m - 1].count)));
            const int jrec = c->last_rec;
            MSC_TRY(read_counter(c, kc, &joined));
            prof_out(c, jrec, (int64_t)joined);
            Cset = B[m];
        }
        // With set capture C_m is built for the dump: a dense bitset over the stage box
        // when pruning bounds the box (one pass), otherwise a hash set sized by a first,
        // counting pass
        const uint64_t box_words = box[m].voxels() * (uint64_t)na * na / 64;
        const bool dense_c = p.prune && !box[m].empty() && box_words <= (1ull << 31);
        uint64_t hits = 1;
        if (!capture) {
            hits = 0;
        } else if (dense_c) {
            MSC_TRY(make_set(c, p, box[m], 0, fast, true, Cset));
        } else {
            unsigned long long* hc = take_counter(c);
            unsigned long long* kc = take_counter(c);
            if (!hc || !kc) return fail(c, MSC_E_CAPACITY, "out of counters");
            LAUNCH(MSC_K_JOIN, m, (int64_t)F[m - 1].count,
                   launch_meet(F[m - 1].list, F[m - 1].count, F[m - 1].view, B[m].view, B[m].view, g, jv[m - 1],
                               kMeetCount, hc, kc, ovf, p.target[0], p.target[1], p.target[2], meet_r2, c->stream));
            MSC_TRY(read_counter(c, hc, &hits));
            if (hits) MSC_TRY(make_set(c, p, box[m], hits, fast, false, Cset));
        }
        if (hits) {
            unsigned long long* cc = take_counter(c);
            unsigned long long* kc2 = take_counter(c);
            if (!cc || !kc2) return fail(c, MSC_E_CAPACITY, "out of counters");
            LAUNCH(MSC_K_JOIN, m, (int64_t)F[m - 1].count,
                   launch_meet(F[m - 1].list, F[m - 1].count, F[m - 1].view, B[m].view, Cset.view, g, jv[m - 1],
                               kMeetInsert, cc, kc2, ovf, p.target[0], p.target[1], p.target[2], meet_r2,
                               c->stream));
            const int jrec = c->last_rec;
            MSC_TRY(read_counter(c, cc, &joined));
            prof_out(c, jrec, (int64_t)joined);
            Cset.count = joined;
        }
    }
    c->stats.join_count = (capture || m == 0) ? (int64_t)joined : -1;
    if (capture && joined) {
        MSC_TRY(capture_set(c, Cset, N, 2, m));
        c->captured[{3, m}] = c->captured[{2, m}];
        if (m >= 1) MSC_TRY(capture_set(c, F[m - 1], N, 3, m - 1));
    }
    if (joined == 0) {
        MSC_TRY(release_top());
        return MSC_NO_REACH;
    }
    for (int k = m - 1; k >= 1; --k) {
        // D_{k-1} from D_k (D_k is Cset for k == m, else F_k's marked structure)
        unsigned long long* dc = take_counter(c);
        int64_t rt_k = 0;
        for (int j = k; j < n; ++j) rt_k += R[j];
        const long long dr2 = p.prune ? (long long)(rt_k * rt_k) : -1;
        LAUNCH(MSC_K_DMARK, k - 1, (int64_t)F[k - 1].count,
               launch_dmark(F[k - 1].list, F[k - 1].count, F[k - 1].view, F[k].view, g, jv[k - 1], dc, p.target[0],
                            p.target[1], p.target[2], dr2, c->stream, shape_for(c, MSC_K_DMARK, F[k - 1].count)));
        if (capture) MSC_TRY(capture_set(c, F[k - 1], N, 3, k - 1));
    }

    // Canonical reach poses.
    void *h_sols, *d_sols, *h_nsol, *d_nsol;
    MSC_TRY(host_area(c, (size_t)want * n * 4, &h_sols, &d_sols));
    MSC_TRY(host_area(c, 4, &h_nsol, &d_nsol));
    *(volatile int32_t*)h_nsol = 0;
    DfsArgs da{};
    for (int k = 0; k <= n; ++k) da.sets[k] = (k < m) ? F[k].view : (k == m ? Cset.view : B[k].view);
    for (int k = 0; k < n; ++k) da.joints[k] = jv[k];
    da.g = g;
    da.n = n;
    da.m = m;
    da.na = na;
    da.want = want;
    for (int k = 0; k < n; ++k) da.ref[k] = p.ref[k];
    da.root = pack_key(p.base[0], p.base[1], p.base[2], p.ia0, p.ie0);
    da.sols = (int32_t*)d_sols;
    da.nsol = (int32_t*)d_nsol;
    LAUNCH(MSC_K_DFS, -1, 0, launch_dfs(da, c->stream));
    MSC_TRY(release_top());   // after the canonical walk, the last reader of the sets
    MSC_TRY(check_overflow(c, ovf, "a stage set"));   // synchronises the stream
    int32_t nsol = *(volatile int32_t*)h_nsol;
    if (nsol <= 0) return fail(c, MSC_E_STATE, "join not empty but no pose traced");
    out.nsol = std::min(nsol, want);
    out.sols.assign((const int32_t*)h_sols, (const int32_t*)h_sols + (size_t)out.nsol * n);
    return MSC_OK;
}

msc_status joint_views(Lane* c, const Plan& p, std::vector<JointView>& jv) {
    jv.resize(p.n);
    for (int k = 0; k < p.n; ++k) {
        TableEntry t;
        MSC_TRY(get_table(c, p.na, p.S, p.len[k], &t));
        jv[k] = JointView{t.off, t.sweep, p.type[k], p.lo[k], p.hi[k], p.S};
    }
    return MSC_OK;
}

msc_status pose_check_steps(Lane* c, const msc_scene* sc, const Plan& p, const int32_t* q_steps, int64_t count,
                            uint8_t* valid, int32_t* ends) {
    std::vector<JointView> jv;
    MSC_TRY(joint_views(c, p, jv));
    PoseArgs a{};
    for (int k = 0; k < p.n; ++k) a.joints[k] = jv[k];
    const size_t qbytes = (size_t)count * p.n * 4, ebytes = (size_t)count * 12;
    if (qbytes + ebytes + (size_t)count + 1024 <= kStagingBytes / 2) {
        // small batch: the kernel reads the poses from and writes the results to mapped
        // host memory
        void *hq, *dq, *hv, *dv, *he = nullptr, *de = nullptr;
        MSC_TRY(host_area(c, qbytes, &hq, &dq));
        MSC_TRY(host_area(c, (size_t)count, &hv, &dv));
        if (ends) MSC_TRY(host_area(c, ebytes, &he, &de));
        std::memcpy(hq, q_steps, qbytes);
        a.g = grid_view(sc);
        a.n = p.n;
        a.na = p.na;
        a.bx = p.base[0];
        a.by = p.base[1];
        a.bz = p.base[2];
        a.ia0 = p.ia0;
        a.ie0 = p.ie0;
        LAUNCH(MSC_K_POSE, -1, count,
               launch_pose_check(a, (const int32_t*)dq, count, (uint8_t*)dv, (int32_t*)de, c->stream));
        MSC_TRY(sync_lane(c));
        std::memcpy(valid, hv, (size_t)count);
        if (ends) std::memcpy(ends, he, ebytes);
        return MSC_OK;
    }
    void *d_q, *d_valid, *d_ends = nullptr;
    MSC_TRY(arena_alloc(c, (uint64_t)count * p.n * 4, &d_q));
    MSC_TRY(arena_alloc(c, (uint64_t)count, &d_valid));
    if (ends) MSC_TRY(arena_alloc(c, (uint64_t)count * 12, &d_ends));
    HIP_TRY(hipMemcpyAsync(d_q, q_steps, qbytes, hipMemcpyHostToDevice, c->stream));
    a.g = grid_view(sc);
    a.n = p.n;
    a.na = p.na;
    a.bx = p.base[0];
    a.by = p.base[1];
    a.bz = p.base[2];
    a.ia0 = p.ia0;
    a.ie0 = p.ie0;
    LAUNCH(MSC_K_POSE, -1, count, launch_pose_check(a, (const int32_t*)d_q, count, (uint8_t*)d_valid, (int32_t*)d_ends, c->stream));
    HIP_TRY(hipMemcpyAsync(valid, d_valid, (size_t)count, hipMemcpyDeviceToHost, c->stream));
    if (ends) HIP_TRY(hipMemcpyAsync(ends, d_ends, (size_t)count * 12, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MSC_OK;
}

msc_status check_scene(Lane* c, const msc_scene* s) {
    if (!s) return fail(c, MSC_E_ARG, "scene is NULL");
    if (s->ctx != c->owner) return fail(c, MSC_E_ARG, "scene belongs to another context");
    if (s->ready && c != c->owner->control && hipStreamWaitEvent(c->stream, s->ready, 0) != hipSuccess)
        return fail(c, MSC_E_HIP, "hipStreamWaitEvent");
    return MSC_OK;
}

msc_opts opts_or_default(const msc_opts* o) {
    msc_opts d;
    msc_opts_default(&d);
    return o ? *o : d;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {

// ---------------------------------------------------------------------------
// Lanes
// ---------------------------------------------------------------------------
constexpr uint64_t kLaneReserved = 64 * 1024;   // counters at the start of each window

msc_status lane_init(Lane* L, msc_ctx* o, int index, hipStream_t stream, bool own, char* base, uint64_t size) {
    L->owner = o;
    L->index = index;
    L->device = o->device;
    L->stream = stream;
    L->own_stream = own;
    if (size <= kLaneReserved + (1u << 20)) return MSC_E_NOMEM;
    L->counters = (unsigned long long*)base;
    L->ws = base + kLaneReserved;
    L->hi = size - kLaneReserved;
    L->lo = 0;
    L->top = 0;
    L->clean = L->hi;
    // coherent: the host polls values that kernels write while the stream runs on
    if (hipHostMalloc((void**)&L->staging, kStagingBytes, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return MSC_E_HIP;
    if (hipHostGetDevicePointer((void**)&L->staging_dev, L->staging, 0) != hipSuccess) return MSC_E_HIP;
    std::memset(L->staging, 0, kStagingBytes);
    L->publish_seq = 0;
    return MSC_OK;
}

void lane_free(Lane* L) {
    if (!L) return;
    (void)hipStreamSynchronize(L->stream);
    if (L->staging) (void)hipHostFree(L->staging);
    for (hipEvent_t e : L->events) (void)hipEventDestroy(e);
    if (L->own_stream) (void)hipStreamDestroy(L->stream);
    delete L;
}

// Split [0, table_lo) into 1 + nworkers equal windows (control lane first).
msc_status layout_lanes(msc_ctx* o, int nworkers) {
    for (Lane* w : o->workers) lane_free(w);
    o->workers.clear();
    const uint64_t total = o->table_lo;
    const uint64_t win = (total / (uint64_t)(nworkers + 1)) & ~(kAlign - 1);
    if (!o->control) {
        o->control = new (std::nothrow) Lane();
        if (!o->control) return MSC_E_NOMEM;
        msc_status st = lane_init(o->control, o, 0, o->stream, false, o->ws, win);
        if (st != MSC_OK) return st;
    } else {
        o->control->counters = (unsigned long long*)o->ws;
        o->control->ws = o->ws + kLaneReserved;
        o->control->hi = win - kLaneReserved;
        o->control->lo = 0;
        o->control->top = 0;
        o->control->clean = o->control->hi;
    }
    for (int i = 0; i < nworkers; ++i) {
        Lane* L = new (std::nothrow) Lane();
        if (!L) return MSC_E_NOMEM;
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            delete L;
            return MSC_E_HIP;
        }
        msc_status r = lane_init(L, o, i + 1, st, true, o->ws + (uint64_t)(i + 1) * win, win);
        o->workers.push_back(L);
        if (r != MSC_OK) return r;
    }
    return MSC_OK;
}

msc_status ctx_fail(msc_ctx* o, msc_status st, const char* msg) {
    if (o) o->err = msg;
    return st;
}

// ---------------------------------------------------------------------------
// One query on one lane
// ---------------------------------------------------------------------------
msc_status reach_on(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t target[3], const msc_opts* opts,
                    int32_t* angles_out) {

    MSC_TRY(check_scene(c, sc));
    MSC_TRY(check_arm(c, arm, sc->n));
    if (!target || !angles_out) return fail(c, MSC_E_ARG, "NULL target or output");
    for (int i = 0; i < 3; ++i)
        if (target[i] < 0 || target[i] >= sc->n) return fail(c, MSC_E_ARG, "target outside the grid");
    msc_opts o = opts_or_default(opts);
    if (o.split_m < -1 || o.split_m > arm->dof) return fail(c, MSC_E_ARG, "split_m outside -1..dof");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    Plan p;
    make_plan(arm, target, p);
    p.prune = (o.flags & MSC_NO_PRUNE) ? 0 : 1;
    p.count_sets = (o.flags & MSC_COUNT_SETS) ? 1 : 0;
    p.split = o.split_m;
    MSC_TRY(set_approach(c, o, p));
    ReachOut r;
    msc_status st = run_reach(c, sc, p, 1, (o.flags & MSC_CAPTURE_SETS) != 0, r);
    if (st != MSC_OK) return st;
    for (int k = 0; k < p.n; ++k) angles_out[k] = r.sols[k] * arm->step_cdeg;
    return MSC_OK;
}

// ref_cdeg (may be null): the original path, (waypoints + 1) * dof centidegrees.  With
// it every one of the first reach_retries reach poses is tried and the path nearest
// the original one is kept (replanning); without it the first path found is returned.
msc_status path_on(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                   const int32_t target[3], int32_t waypoints, int32_t max_delta_cdeg, const msc_opts* opts,
                   int32_t* path_out, const int32_t* ref_cdeg = nullptr) {

    MSC_TRY(check_scene(c, sc));
    MSC_TRY(check_arm(c, arm, sc->n));
    if (!start_cdeg || !target || !path_out) return fail(c, MSC_E_ARG, "NULL argument");
    for (int i = 0; i < 3; ++i)
        if (target[i] < 0 || target[i] >= sc->n) return fail(c, MSC_E_ARG, "target outside the grid");
    if (waypoints < 0 || waypoints > 4096) return fail(c, MSC_E_ARG, "waypoints outside 0..4096");
    if (max_delta_cdeg <= 0 || max_delta_cdeg % arm->step_cdeg)
        return fail(c, MSC_E_ARG, "max_delta must be a positive multiple of the step");
    msc_opts o = opts_or_default(opts);
    if (o.tube_r0 < 0 || o.tube_r1 < 0 || o.reach_retries < 1 || o.reach_retries > 64)
        return fail(c, MSC_E_ARG, "bad options");
    if (o.split_m < -1 || o.split_m > arm->dof) return fail(c, MSC_E_ARG, "split_m outside -1..dof");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    Plan p;
    make_plan(arm, target, p);
    p.prune = (o.flags & MSC_NO_PRUNE) ? 0 : 1;
    p.count_sets = (o.flags & MSC_COUNT_SETS) ? 1 : 0;
    p.split = o.split_m;
    MSC_TRY(set_approach(c, o, p));
    const int n = p.n;
    const int delta = max_delta_cdeg / arm->step_cdeg;
    int start[kMaxDof];
    for (int k = 0; k < n; ++k) {
        if (start_cdeg[k] % arm->step_cdeg) return fail(c, MSC_E_ARG, "start angle %d not a multiple of the step", k);
        start[k] = start_cdeg[k] / arm->step_cdeg;
        if (start[k] < p.lo[k] || start[k] > p.hi[k]) return fail(c, MSC_E_ARG, "start angle %d outside its limits", k);
    }
    std::vector<int32_t> ref;
    if (ref_cdeg) {
        ref.assign(ref_cdeg, ref_cdeg + (size_t)(waypoints + 1) * n);
        for (auto& v : ref) {
            if (v % arm->step_cdeg) return fail(c, MSC_E_ARG, "reference path angle not a multiple of the step");
            v /= arm->step_cdeg;
        }
    }
    uint8_t ok = 0;
    MSC_TRY(pose_check_steps(c, sc, p, start, 1, &ok, nullptr));
    if (!ok) return fail(c, MSC_E_ARG, "start pose is not clear of obstacles");
    begin_call(c);
    int lim_lo[kMaxDof], lim_hi[kMaxDof];
    for (int k = 0; k < n; ++k) {
        lim_lo[k] = p.lo[k];
        lim_hi[k] = p.hi[k];
        int64_t span = (int64_t)waypoints * delta;
        p.lo[k] = (int)std::max<int64_t>(p.lo[k], start[k] - span);
        p.hi[k] = (int)std::min<int64_t>(p.hi[k], start[k] + span);
        p.ref[k] = start[k];
    }
    ReachOut r;
    msc_status st = run_reach(c, sc, p, o.reach_retries, (o.flags & MSC_CAPTURE_SETS) != 0, r);
    if (st != MSC_OK) return st;
    c->stats.attempts = 0;
    if (waypoints == 0) {
        for (int k = 0; k < n; ++k) path_out[k] = start[k] * arm->step_cdeg;
        return MSC_OK;
    }
    std::vector<JointView> jv;
    for (int k = 0; k < n; ++k) {
        p.lo[k] = lim_lo[k];
        p.hi[k] = lim_hi[k];
    }
    MSC_TRY(joint_views(c, p, jv));
    const uint64_t mark = c->lo;
    const size_t stage_mark = c->staging_used;
    const int radii[2] = {o.tube_r0, o.tube_r1};
    const int nr = o.tube_r1 == o.tube_r0 ? 1 : 2;
    const int nsol = r.nsol;
    if (nsol < 1) return MSC_NO_PATH;
    const size_t rows = (size_t)(waypoints + 1) * n;
    // The attempts in search order: reach pose i at radius index ri is attempt i * nr + ri.
    // res: -1 not searched, 0 no path, 1 a path (kept in found).
    std::vector<int8_t> res((size_t)nsol * nr, -1);
    std::vector<std::vector<int32_t>> found((size_t)nsol * nr);
    auto tube_args = [&](int rad, int pose, TubeArgs& ta) -> msc_status {
        uint64_t slab = 1;
        for (int k = 0; k < n; ++k) {
            slab *= (uint64_t)(2 * rad + 1);
            if (slab > (1ull << 28)) return fail(c, MSC_E_CAPACITY, "tube of radius %d too large", rad);
        }
        ta = TubeArgs{};
        for (int k = 0; k < n; ++k) ta.joints[k] = jv[k];
        ta.g = grid_view(sc);
        ta.n = n;
        ta.na = p.na;
        ta.bx = p.base[0];
        ta.by = p.base[1];
        ta.bz = p.base[2];
        ta.ia0 = p.ia0;
        ta.ie0 = p.ie0;
        ta.W = waypoints;
        ta.delta = delta;
        ta.r = rad;
        for (int k = 0; k < n; ++k) {
            ta.start[k] = start[k];
            ta.goal[k] = r.sols[(size_t)pose * n + k];
            ta.lim_lo[k] = lim_lo[k];
            ta.lim_hi[k] = lim_hi[k];
        }
        ta.slab = slab;
        return MSC_OK;
    };
    // A group of attempts: the tubes toward the reach poses `poses` at radius index ri.
    // In the blocked layout the attempts of a group differ only in their goal, so they
    // run at once, one block each; each is the search a lone attempt would make.
    struct Group {
        int ri = 0;
        std::vector<int> poses;
        int32_t* h_path = nullptr;
        int32_t* h_status = nullptr;
    };
    // Launches a group (ok = false, nothing allocated, when a group of several attempts
    // does not fit the lane's workspace or staging buffer).
    auto launch_group = [&](Group& gr, bool& ok) -> msc_status {
        const hipStream_t stream = c->stream;
        ok = true;
        const int rad = radii[gr.ri];
        const int A = (int)gr.poses.size();
        TubeArgs ta;
        MSC_TRY(tube_args(rad, gr.poses[0], ta));
        const TubeBlk tb = tube_blk_plan(ta);
        const uint64_t words = (uint64_t)(waypoints + 1) * tb.nw;   // one attempt's frames
        if (A > 1) {
            const size_t host = 4 * 256 + (size_t)A * (rows * 4 + 4 + 2 * (size_t)n * 4);
            ok = tb.lds && 2 * words * 8 * (uint64_t)A + ((uint64_t)A * n * 4 + 4096) <= free_bytes(c) &&
                 c->staging_used + host + 4096 <= kStagingBytes;
            if (!ok) return MSC_OK;
        }
        void *h_path, *d_path, *h_status, *d_status;
        MSC_TRY(host_area(c, (size_t)A * rows * 4, &h_path, &d_path));
        MSC_TRY(host_area(c, (size_t)A * 4, &h_status, &d_status));
        gr.h_path = (int32_t*)h_path;
        gr.h_status = (int32_t*)h_status;
        for (int i = 0; i < A; ++i) ((volatile int32_t*)h_status)[i] = 0;
        const uint64_t cells = (uint64_t)(waypoints + 1) * ta.slab;
        if (tb.lds) {
            // frames that fit LDS: bit-parallel search in one block per attempt
            const int32_t* d_goals = nullptr;
            if (A > 1) {
                std::vector<int32_t> goals((size_t)A * n);
                for (int i = 0; i < A; ++i)
                    for (int k = 0; k < n; ++k) goals[(size_t)i * n + k] = r.sols[(size_t)gr.poses[i] * n + k];
                void *hg, *hgd, *dg;
                MSC_TRY(host_area(c, goals.size() * 4, &hg, &hgd));
                std::memcpy(hg, goals.data(), goals.size() * 4);
                MSC_TRY(arena_alloc(c, goals.size() * 4, &dg));
                HIP_TRY(hipMemcpyAsync(dg, hg, goals.size() * 4, hipMemcpyHostToDevice, stream));
                d_goals = (const int32_t*)dg;
            }
            void *d_vbits, *d_rbits;
            MSC_TRY(arena_alloc(c, words * 8 * (uint64_t)A, &d_vbits));
            MSC_TRY(arena_alloc(c, words * 8 * (uint64_t)A, &d_rbits));
            LAUNCH(MSC_K_TUBE_SOLVE, rad, (int64_t)cells * A,
                   launch_tube_bits(ta, tb, (uint64_t*)d_vbits, (uint64_t*)d_rbits, (int32_t*)d_path,
                                    (int32_t*)d_status, stream, A, d_goals));
        } else {
            void *d_valid, *d_reach, *d_t0, *d_t1;
            MSC_TRY(arena_alloc(c, cells, &d_valid));
            MSC_TRY(arena_alloc(c, cells, &d_reach));
            MSC_TRY(arena_alloc(c, ta.slab, &d_t0));
            MSC_TRY(arena_alloc(c, ta.slab, &d_t1));
            LAUNCH(MSC_K_TUBE_VALID, rad, (int64_t)cells, launch_tube_valid(ta, (uint8_t*)d_valid, stream));
            LAUNCH(MSC_K_TUBE_SOLVE, rad, (int64_t)cells,
                   launch_tube_solve(ta, (const uint8_t*)d_valid, (uint8_t*)d_reach, (uint8_t*)d_t0,
                                     (uint8_t*)d_t1, (int32_t*)d_path, (int32_t*)d_status, stream));
        }
        return MSC_OK;
    };
    auto collect = [&](const Group& gr) {
        for (size_t i = 0; i < gr.poses.size(); ++i) {
            const size_t at = (size_t)gr.poses[i] * nr + gr.ri;
            res[at] = ((volatile int32_t*)gr.h_status)[i] ? 1 : 0;
            if (res[at]) {
                const int32_t* src = gr.h_path + i * rows;
                found[at].assign(src, src + rows);
            }
        }
    };
    // Runs the groups of one phase on the lane's stream with one wait for all (a second
    // stream per lane would share the few hardware queues with the other lanes' streams);
    // when the groups do not all fit, their attempts one at a time, as lone attempts.
    auto phase = [&](std::vector<Group> groups) -> msc_status {
        c->lo = mark;
        c->staging_used = stage_mark;
        std::vector<Group*> live;
        for (Group& gr : groups)
            if (!gr.poses.empty()) live.push_back(&gr);
        bool all = true;
        for (size_t g = 0; g < live.size() && all; ++g) MSC_TRY(launch_group(*live[g], all));
        MSC_TRY(sync_lane(c));   // also what was launched before a group did not fit
        if (all) {
            for (Group* gr : live) collect(*gr);
            return MSC_OK;
        }
        for (Group* gr : live)
            for (int pose : gr->poses) {
                c->lo = mark;
                c->staging_used = stage_mark;
                Group one;
                one.ri = gr->ri;
                one.poses = {pose};
                bool ok;
                MSC_TRY(launch_group(one, ok));
                MSC_TRY(sync_lane(c));
                collect(one);
            }
        return MSC_OK;
    };
    auto group = [](int ri, std::vector<int> poses) {
        Group g;
        g.ri = ri;
        g.poses = std::move(poses);
        return g;
    };
    auto succeeded = [&](int pose, int ri) { return res[(size_t)pose * nr + ri] == 1; };
    int win_pose = -1, win_ri = -1;
    // A lone query on the control lane has the device to itself: after a failed first
    // attempt every other attempt is searched in one phase.  A worker lane shares the
    // device with the other lanes, so it runs no more attempts than the search order can
    // need: the first radius of the other poses and the first pose's second radius, then
    // the second radius of the poses before the first pose whose first radius gave a path.
    const bool eager = c == c->owner->control;
    std::vector<int> rest, every;
    for (int i = 1; i < nsol; ++i) rest.push_back(i);
    for (int i = 0; i < nsol; ++i) every.push_back(i);
    if (ref.empty()) {
        // the first path in search order
        MSC_TRY(phase({group(0, {0})}));
        if (!succeeded(0, 0) && (nsol > 1 || nr > 1)) {
            std::vector<Group> ga{group(0, rest)};
            if (nr > 1) ga.push_back(group(1, eager ? every : std::vector<int>{0}));
            MSC_TRY(phase(ga));
            if (!eager && nr > 1 && !succeeded(0, 1)) {
                std::vector<int> second;
                for (int i = 1; i < nsol && !succeeded(i, 0); ++i) second.push_back(i);
                MSC_TRY(phase({group(1, second)}));
            }
        }
        int tried = 0;
        for (int i = 0; i < nsol && win_pose < 0; ++i)
            for (int ri = 0; ri < nr; ++ri) {
                ++tried;
                if (succeeded(i, ri)) {
                    win_pose = i;
                    win_ri = ri;
                    break;
                }
            }
        c->stats.attempts = tried;
        if (win_pose < 0) return MSC_NO_PATH;
        const std::vector<int32_t>& path = found[(size_t)win_pose * nr + win_ri];
        for (size_t j = 0; j < path.size(); ++j) path_out[j] = path[j] * arm->step_cdeg;
        c->stats.tube_r = radii[win_ri];
        c->stats.reach_index = win_pose;
        return MSC_OK;
    }
    // Replanning: every reach pose is tried (its first radius with a path counts) and the
    // path nearest the original one is kept, by the sum over the waypoints of the L1
    // distance (steps); the earlier reach pose keeps a tie.  The first radius of every pose
    // is searched in one phase, then the second radius of the poses where it is needed
    // (on any lane: most poses have a path at the first radius, and the second radius
    // costs several times as much).
    MSC_TRY(phase({group(0, every)}));
    if (nr > 1) {
        std::vector<int> second;
        for (int i = 0; i < nsol; ++i)
            if (!succeeded(i, 0)) second.push_back(i);
        MSC_TRY(phase({group(1, second)}));
    }
    int64_t best_cost = -1;
    int tried = 0;
    for (int i = 0; i < nsol; ++i) {
        for (int ri = 0; ri < nr; ++ri) {
            ++tried;
            if (!succeeded(i, ri)) continue;
            const std::vector<int32_t>& path = found[(size_t)i * nr + ri];
            int64_t cost = 0;
            for (size_t j = 0; j < path.size(); ++j) cost += std::abs((int64_t)path[j] - ref[j]);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                win_pose = i;
                win_ri = ri;
            }
            break;
        }
    }
    c->stats.attempts = tried;
    if (win_pose < 0) return MSC_NO_PATH;
    const std::vector<int32_t>& best = found[(size_t)win_pose * nr + win_ri];
    for (size_t j = 0; j < best.size(); ++j) path_out[j] = best[j] * arm->step_cdeg;
    c->stats.tube_r = radii[win_ri];
    c->stats.reach_index = win_pose;
    return MSC_OK;
}

// ---------------------------------------------------------------------------
// Workspace-guided paths: candidate solutions from the reach search, then one block
// walks the waypoints of each in turn (k_track).
// ---------------------------------------------------------------------------
msc_status track_params(Lane* c, const msc_arm* arm, const msc_track* tr, int default_tracked, TrackArgs& ta) {
    msc_track t;
    msc_track_default(&t);
    if (tr) t = *tr;
    const int step = arm->step_cdeg;
    ta.tracked = t.tracked < 0 ? default_tracked : t.tracked;
    if (ta.tracked < 1 || ta.tracked > arm->dof) return fail(c, MSC_E_ARG, "tracked joint outside 1..dof");
    const int d = t.max_delta_cdeg < 0 ? step : t.max_delta_cdeg;
    const int d2 = t.relaxed_delta_cdeg < 0 ? 2 * step : t.relaxed_delta_cdeg;
    if (d % step || d2 % step || d < 0 || d2 < d)
        return fail(c, MSC_E_ARG, "track deltas must be multiples of the step with 0 <= max <= relaxed");
    ta.delta = d / step;
    ta.delta2 = d2 / step;
    double cells = std::pow(2.0 * ta.delta2 + 1.0, (double)arm->dof);
    if (cells >= 4398046511104.0) return fail(c, MSC_E_ARG, "relaxed joint box has 2^42 poses or more");
    if (t.eps2_vox < 0 || t.eps2_vox > 1023) return fail(c, MSC_E_ARG, "eps2_vox outside 0..1023");
    ta.eps2 = t.eps2_vox;
    return MSC_OK;
}

// Fills the real arm's part of ta (joint views, limits, base) from plan p.
msc_status track_arm(Lane* c, const msc_scene* sc, const Plan& p, TrackArgs& ta) {
    std::vector<JointView> jv;
    MSC_TRY(joint_views(c, p, jv));
    for (int k = 0; k < p.n; ++k) {
        ta.joints[k] = jv[k];
        ta.len[k] = p.len[k];
        ta.lim_lo[k] = p.lo[k];
        ta.lim_hi[k] = p.hi[k];
    }
    ta.g = grid_view(sc);
    ta.n = p.n;
    ta.na = p.na;
    ta.bx = p.base[0];
    ta.by = p.base[1];
    ta.bz = p.base[2];
    ta.ia0 = p.ia0;
    ta.ie0 = p.ie0;
    return MSC_OK;
}

// Runs k_track over the candidate solutions sols[nsol * width] and copies the rows.
msc_status track_run(Lane* c, TrackArgs& ta, const std::vector<int32_t>& sols, int nsol, int width, int max_rows,
                     int step_cdeg, int32_t* path_out, int32_t* rows_out) {
    void *h_sols, *d_sols, *h_rows, *d_rows, *h_st, *d_st;
    MSC_TRY(host_area(c, (size_t)nsol * width * 4, &h_sols, &d_sols));
    MSC_TRY(host_area(c, (size_t)max_rows * ta.n * 4, &h_rows, &d_rows));
    MSC_TRY(host_area(c, 16, &h_st, &d_st));
    std::memcpy(h_sols, sols.data(), (size_t)nsol * width * 4);
    ta.nsol = nsol;
    ta.sols = (const int32_t*)d_sols;
    ta.rows = (int32_t*)d_rows;
    ta.status = (int32_t*)d_st;
    LAUNCH(MSC_K_TRACK, -1, nsol, launch_track(ta, c->stream));
    MSC_TRY(sync_lane(c));
    const volatile int32_t* st = (const volatile int32_t*)h_st;
    const int rows = st[0];
    c->stats.attempts = st[1] < 0 ? nsol : st[1] + 1;
    c->stats.reach_index = st[1];
    if (rows <= 0) return MSC_NO_PATH;
    if (rows > max_rows) return fail(c, MSC_E_CAPACITY, "tracked path longer than planned");
    const int32_t* hr = (const int32_t*)h_rows;
    for (size_t j = 0; j < (size_t)rows * ta.n; ++j) path_out[j] = hr[j] * step_cdeg;
    *rows_out = rows;
    return MSC_OK;
}

// A tracking launch waiting for its query's search: the kernel arguments, the
// candidate solutions and the output sizes.
struct TrackJob {
    TrackArgs ta{};
    std::vector<int32_t> sols;
    int nsol = 0, width = 0, max_rows = 0, step = 0;
};

// The reach search of a reach-pose-guided path; MSC_OK leaves the tracking in job.
msc_status guided_prepare(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t target[3],
                          const msc_track* tr, const msc_opts* opts, TrackJob& job) {
    MSC_TRY(check_scene(c, sc));
    MSC_TRY(check_arm(c, arm, sc->n));
    if (!target) return fail(c, MSC_E_ARG, "NULL target");
    for (int i = 0; i < 3; ++i)
        if (target[i] < 0 || target[i] >= sc->n) return fail(c, MSC_E_ARG, "target outside the grid");
    msc_opts o = opts_or_default(opts);
    if (o.split_m < -1 || o.split_m > arm->dof) return fail(c, MSC_E_ARG, "split_m outside -1..dof");
    if (o.reach_retries < 1 || o.reach_retries > 64) return fail(c, MSC_E_ARG, "bad options");
    TrackArgs& ta = job.ta;
    ta = TrackArgs{};
    MSC_TRY(track_params(c, arm, tr, std::max(1, arm->dof - 2), ta));
    job.max_rows = arm->samples * (ta.tracked - 1) + 1;
    if (job.max_rows > kTrackMaxPoints) return fail(c, MSC_E_ARG, "more than %d waypoints", kTrackMaxPoints);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    Plan p;
    make_plan(arm, target, p);
    p.prune = (o.flags & MSC_NO_PRUNE) ? 0 : 1;
    p.count_sets = (o.flags & MSC_COUNT_SETS) ? 1 : 0;
    p.split = o.split_m;
    MSC_TRY(set_approach(c, o, p));
    ReachOut r;
    msc_status st = run_reach(c, sc, p, o.reach_retries, (o.flags & MSC_CAPTURE_SETS) != 0, r);
    if (st != MSC_OK) return st;
    MSC_TRY(track_arm(c, sc, p, ta));
    ta.mode = 0;
    job.sols = std::move(r.sols);
    job.nsol = r.nsol;
    job.width = p.n;
    job.step = arm->step_cdeg;
    return MSC_OK;
}

// The virtual arm's reach search of a path between poses; MSC_OK leaves the tracking in job.
msc_status pose_path_prepare(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                             const int32_t target[3], const msc_arm* varm, const msc_track* tr,
                             const msc_opts* opts, TrackJob& job) {
    MSC_TRY(check_scene(c, sc));
    MSC_TRY(check_arm(c, arm, sc->n));
    if (!start_cdeg || !target || !varm) return fail(c, MSC_E_ARG, "NULL argument");
    for (int i = 0; i < 3; ++i)
        if (target[i] < 0 || target[i] >= sc->n) return fail(c, MSC_E_ARG, "target outside the grid");
    if (varm->step_cdeg != arm->step_cdeg) return fail(c, MSC_E_ARG, "the virtual arm's step differs from the arm's");
    msc_opts o = opts_or_default(opts);
    if (o.split_m < -1 || o.reach_retries < 1 || o.reach_retries > 64) return fail(c, MSC_E_ARG, "bad options");
    TrackArgs& ta = job.ta;
    ta = TrackArgs{};
    MSC_TRY(track_params(c, arm, tr, arm->dof, ta));
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    Plan p;
    make_plan(arm, target, p);
    int start[kMaxDof];
    for (int k = 0; k < p.n; ++k) {
        if (start_cdeg[k] % arm->step_cdeg) return fail(c, MSC_E_ARG, "start angle %d not a multiple of the step", k);
        start[k] = start_cdeg[k] / arm->step_cdeg;
        if (start[k] < p.lo[k] || start[k] > p.hi[k]) return fail(c, MSC_E_ARG, "start angle %d outside its limits", k);
        ta.start[k] = start[k];
    }
    uint8_t ok = 0;
    MSC_TRY(pose_check_steps(c, sc, p, start, 1, &ok, nullptr));
    if (!ok) return fail(c, MSC_E_ARG, "start pose is not clear of obstacles");
    // the virtual arm's root: joint `tracked` of the start pose
    Plan ps = p;
    ps.n = ta.tracked;
    int32_t root[3];
    MSC_TRY(pose_check_steps(c, sc, ps, start, 1, &ok, root));
    msc_arm va = *varm;
    for (int i = 0; i < 3; ++i) va.base[i] = root[i];
    MSC_TRY(check_arm(c, &va, sc->n));
    job.max_rows = va.samples * va.dof + 1;
    if (job.max_rows > kTrackMaxPoints) return fail(c, MSC_E_ARG, "more than %d waypoints", kTrackMaxPoints);
    begin_call(c);
    Plan pv;
    make_plan(&va, target, pv);
    pv.prune = (o.flags & MSC_NO_PRUNE) ? 0 : 1;
    pv.split = o.split_m > va.dof ? -1 : o.split_m;
    ReachOut r;
    msc_status st = run_reach(c, sc, pv, o.reach_retries, false, r);
    if (st != MSC_OK) return st;
    std::vector<JointView> vjv;
    MSC_TRY(joint_views(c, pv, vjv));
    for (int k = 0; k < pv.n; ++k) {
        ta.vjoints[k] = vjv[k];
        ta.vlen[k] = pv.len[k];
    }
    ta.vn = pv.n;
    ta.vbx = pv.base[0];
    ta.vby = pv.base[1];
    ta.vbz = pv.base[2];
    ta.via0 = pv.ia0;
    ta.vie0 = pv.ie0;
    MSC_TRY(track_arm(c, sc, p, ta));
    ta.mode = 1;
    job.sols = std::move(r.sols);
    job.nsol = r.nsol;
    job.width = pv.n;
    job.step = arm->step_cdeg;
    return MSC_OK;
}

// The short-reach shortcut ("Short Reaches") of plan p on its own forward sets
// F_0..F_{K-1} (the hit search marks them in place, so they are not the reach search's):
// *found = 0 without a hit, else q[0..k) (steps), k, the hit sample and the length.
struct ShortcutHit {
    int found = 0, k = 0, s = 0;
    long long length = 0;
    int q[kMaxDof] = {};
};

msc_status shortcut_search(Lane* c, const msc_scene* sc, const Plan& p, int K, int rho2, ShortcutHit& hit) {
    const int n = p.n, na = p.na, N = sc->n;
    const GridView g = grid_view(sc);
    hit = ShortcutHit();
    LAUNCH(MSC_K_FILL, -1, 0, launch_fill((uint64_t*)c->counters, kCounters, 0ull, c->stream));
    c->ovf = take_counter(c);
    std::vector<JointView> jv(n);
    std::vector<int64_t> R(n);
    for (int k = 0; k < n; ++k) {
        TableEntry t;
        MSC_TRY(get_table(c, na, p.S, p.len[k], &t));
        jv[k] = JointView{t.off, t.sweep, p.type[k], p.lo[k], p.hi[k], p.S};
        R[k] = isqrt_ceil((int64_t)t.maxn2);
    }
    std::vector<StageSet> F(K);
    {
        Box b0{p.base[0], p.base[1], p.base[2], 1, 1, 1};
        MSC_TRY(make_set(c, p, b0, 1, 0, false, F[0]));
        void* l0;
        MSC_TRY(arena_alloc(c, 8, &l0));
        unsigned long long* ctr = take_counter(c);
        if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
        LAUNCH(MSC_K_SEED, 0, 0,
               launch_seed_fwd(F[0].view, g, p.base[0], p.base[1], p.base[2], p.ia0, p.ie0, (uint64_t*)l0, ctr,
                               c->stream));
        MSC_TRY(read_counter(c, ctr, &F[0].count));
        F[0].list = (uint64_t*)l0;
        F[0].listed = true;
    }
    std::vector<long long> r2s(K, -1);
    for (int k = 1; k < K && F[k - 1].count; ++k) {
        MSC_TRY(ensure_list(c, F[k - 1]));
        const uint64_t upper = F[k - 1].count * (uint64_t)(p.hi[k - 1] - p.lo[k - 1] + 1);
        const int fast = p.type[k] == MSC_YAW ? 1 : 0;
        MSC_TRY(make_set(c, p, stage_box(p, N, R, k), upper, fast, false, F[k]));
        int64_t rt = 0;
        for (int j = k; j < n; ++j) rt += R[j];
        r2s[k] = p.prune ? (long long)(rt * rt) : -1;
        unsigned long long* ctr = take_counter(c);
        if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
        LAUNCH(MSC_K_EXPAND_FWD, k, (int64_t)F[k - 1].count,
               launch_expand_fwd(F[k - 1].list, F[k - 1].count, F[k].view, g, jv[k - 1], p.target[0], p.target[1],
                                 p.target[2], r2s[k], ctr, c->ovf, c->stream,
                                 shape_for(c, MSC_K_EXPAND_FWD, F[k - 1].count)));
        MSC_TRY(read_counter(c, ctr, &F[k].count));
    }
    MSC_TRY(check_overflow(c, c->ovf, "a stage set of the shortcut search"));
    for (int k = 1; k < K; ++k)
        if (F[k].count) MSC_TRY(ensure_list(c, F[k]));
    // the least hit key over segments 2..K
    unsigned long long* best = take_counter(c);
    if (!best) return fail(c, MSC_E_CAPACITY, "out of counters");
    HIP_TRY(launch_fill((uint64_t*)best, 1, ~0ull, c->stream));
    std::vector<HitArgs> ha(K + 1);
    long long base_len = 0;
    for (int k = 1; k <= K; ++k) {
        HitArgs& h = ha[k];
        h = HitArgs{};
        h.g = g;
        h.na = na;
        h.tx = p.target[0];
        h.ty = p.target[1];
        h.tz = p.target[2];
        h.rho2 = rho2;
        h.k = k;
        h.base_len = base_len;
        h.len = p.len[k - 1];
        base_len += (long long)p.S * p.len[k - 1];
        if (k >= 2 && F[k - 1].count)
            LAUNCH(MSC_K_JOIN, k, (int64_t)F[k - 1].count,
                   launch_hits(F[k - 1].list, F[k - 1].count, jv[k - 1], h, best, c->stream));
    }
    uint64_t key = 0;
    MSC_TRY(read_counter(c, best, &key));
    if (key == ~0ull) return MSC_OK;
    const int k = (int)((key >> 16) & 0xff);
    // D_{k-1}: the states with a best hit; D_{j-1} from D_j back to the root
    LAUNCH(MSC_K_DMARK, k - 1, (int64_t)F[k - 1].count,
           launch_hit_mark(F[k - 1].list, F[k - 1].count, F[k - 1].view, jv[k - 1], ha[k], best, c->stream));
    for (int j = k - 1; j >= 1; --j) {
        unsigned long long* dc = take_counter(c);
        if (!dc) return fail(c, MSC_E_CAPACITY, "out of counters");
        LAUNCH(MSC_K_DMARK, j - 1, (int64_t)F[j - 1].count,
               launch_dmark(F[j - 1].list, F[j - 1].count, F[j - 1].view, F[j].view, g, jv[j - 1], dc, p.target[0],
                            p.target[1], p.target[2], r2s[j], c->stream));
    }
    HitWalkArgs wa{};
    for (int j = 1; j < k; ++j) wa.D[j] = F[j].view;
    for (int j = 0; j < k; ++j) wa.joints[j] = jv[j];
    wa.h = ha[k];
    wa.na = na;
    wa.bx = p.base[0];
    wa.by = p.base[1];
    wa.bz = p.base[2];
    wa.ia0 = p.ia0;
    wa.ie0 = p.ie0;
    wa.best = best;
    void *h_out, *d_out;
    MSC_TRY(host_area(c, (kMaxDof + 1) * 4, &h_out, &d_out));
    wa.out = (int32_t*)d_out;
    LAUNCH(MSC_K_DFS, -1, 0, launch_hit_walk(wa, c->stream));
    MSC_TRY(sync_lane(c));
    const volatile int32_t* ho = (const volatile int32_t*)h_out;
    if (ho[kMaxDof] <= 0) return fail(c, MSC_E_STATE, "the shortcut walk found no move");
    hit.found = 1;
    hit.k = k;
    hit.s = ho[kMaxDof];
    hit.length = (long long)(key >> 40);
    for (int j = 0; j < k; ++j) hit.q[j] = ho[j];
    return MSC_OK;
}

// ---------------------------------------------------------------------------
// The paper's gap search: the quiver on the host (FP64, the platform's libm), the
// search in the gMS kernels.
// ---------------------------------------------------------------------------
double gms_rad(double deg) { return (deg * M_PI) / 180.0; }

long long gms_round_host(double v) {
    const double a = std::fabs(v);
    const double f = std::floor(a);
    const double frac = a - f;
    const double r = (frac > 0.5 || std::fabs(frac - 0.5) <= 1e-9) ? f + 1.0 : f;
    return v >= 0 ? (long long)r : -(long long)r;
}

bool build_quiver(int step_cdeg, int min_ring, std::vector<double>& Q) {
    Q.clear();
    // steps below 0.2 degrees would give 2^20 vectors or more
    if (step_cdeg < 20 || 18000 % step_cdeg || min_ring < 1) return false;
    const double D = step_cdeg / 100.0;
    const int n = 36000 / step_cdeg;
    for (int i = 0; i <= 18000 / step_cdeg; ++i) {
        const double e = -90.0 + i * D;
        int m = 1;
        if (std::fabs(e) != 90.0) m = std::max<long long>(min_ring, gms_round_host(n * std::cos(gms_rad(e))));
        const double ce = std::cos(gms_rad(e)), se = std::sin(gms_rad(e));
        for (int j = 0; j < m; ++j) {
            const double a = (j * 360.0) / m;
            Q.push_back(ce * std::cos(gms_rad(a)));
            Q.push_back(ce * std::sin(gms_rad(a)));
            Q.push_back(se);
        }
    }
    return true;
}

// Solutions whose keys are copied to the host and ordered there without a second pass.
constexpr uint64_t kGmsFewKeys = 1u << 16;

msc_status gms_on(Lane* c, const msc_scene* sc, const msc_gms_arm* arm, const int32_t target[3], int32_t want,
                  bool first_only, int64_t* count_out, int32_t* sols_out, double* vec_out, int32_t* nsol_out) {
    MSC_TRY(check_scene(c, sc));
    if (!arm || !target || !count_out || !sols_out || !vec_out || !nsol_out) return fail(c, MSC_E_ARG, "NULL argument");
    if (want < 1) return fail(c, MSC_E_ARG, "want < 1");
    if (arm->samples < 1 || arm->samples > 64) return fail(c, MSC_E_ARG, "samples outside 1..64");
    for (int k = 0; k < 4; ++k)
        if (!(arm->len[k] > 0) || !std::isfinite(arm->len[k])) return fail(c, MSC_E_ARG, "segment length");
    if (!(arm->eps >= 0) || !std::isfinite(arm->eps)) return fail(c, MSC_E_ARG, "eps");
    for (int k = 0; k < 3; ++k)
        if (arm->max_flex_cdeg[k] < 0 || arm->max_flex_cdeg[k] > 18000) return fail(c, MSC_E_ARG, "flexion limit");
    if (arm->approach_half_cdeg > 18000) return fail(c, MSC_E_ARG, "approach half-angle");
    for (int i = 0; i < 3; ++i) {
        if (target[i] < 0 || target[i] >= sc->n) return fail(c, MSC_E_ARG, "target outside the grid");
        if (arm->base[i] < 0 || arm->base[i] >= sc->n) return fail(c, MSC_E_ARG, "base outside the grid");
    }
    std::vector<double> Q;
    if (!build_quiver(arm->step_cdeg, arm->min_ring, Q)) return fail(c, MSC_E_ARG, "bad quiver step or min_ring");
    const int nq = (int)(Q.size() / 3);
    if (nq >= (1 << 20)) return fail(c, MSC_E_ARG, "quiver of 2^20 vectors or more");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    GmsArgs a{};
    a.g = grid_view(sc);
    a.nq = nq;
    a.L1 = arm->len[0];
    a.L2 = arm->len[1];
    a.L3 = arm->len[2];
    a.L4 = arm->len[3];
    for (int i = 0; i < 3; ++i) {
        a.p0[i] = (double)arm->base[i];
        a.t[i] = (double)target[i];
    }
    a.S = arm->samples;
    for (int s = 1; s <= a.S; ++s) a.ts[s - 1] = (double)s / a.S;
    a.min_el = std::sin(gms_rad(arm->seg1_min_el_cdeg / 100.0)) - 1e-9;
    a.c1 = std::cos(gms_rad(arm->max_flex_cdeg[0] / 100.0)) - 1e-9;
    a.c2 = std::cos(gms_rad(arm->max_flex_cdeg[1] / 100.0)) - 1e-9;
    a.c3 = std::cos(gms_rad(arm->max_flex_cdeg[2] / 100.0)) - 1e-9;
    a.has_cone = arm->approach_half_cdeg >= 0;
    if (a.has_cone) {
        const double az = gms_rad(arm->approach_az_cdeg / 100.0), el = gms_rad(arm->approach_el_cdeg / 100.0);
        a.ax[0] = std::cos(el) * std::cos(az);
        a.ax[1] = std::cos(el) * std::sin(az);
        a.ax[2] = std::sin(el);
        a.cone_c = std::cos(gms_rad(arm->approach_half_cdeg / 100.0)) - 1e-9;
    }
    const double r5 = a.L2 + a.L3 + a.L4 + arm->eps, r7 = a.L3 + a.L4 + arm->eps;
    a.r5sq = r5 * r5;
    a.r7sq = r7 * r7;
    const double glo = std::max(a.L3 - arm->eps, 0.0), ghi = a.L3 + arm->eps;
    a.glo = glo * glo;
    a.ghi = ghi * ghi;
    void *d_q, *d_flags;
    MSC_TRY(arena_alloc(c, Q.size() * 8, &d_q));
    HIP_TRY(hipMemcpyAsync(d_q, Q.data(), Q.size() * 8, hipMemcpyHostToDevice, c->stream));
    a.Q = (const double*)d_q;
    MSC_TRY(arena_alloc(c, 2 * (uint64_t)nq, &d_flags));
    LAUNCH(MSC_K_SEED, 0, nq, launch_gms_flags(a, (uint8_t*)d_flags, (uint8_t*)d_flags + nq, c->stream));
    std::vector<uint8_t> flags(2 * (size_t)nq);
    HIP_TRY(hipMemcpyAsync(flags.data(), d_flags, flags.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<int32_t> s1, s4;
    for (int q = 0; q < nq; ++q) {
        if (flags[q]) s1.push_back(q);
        if (flags[nq + q]) s4.push_back(q);
    }
    *count_out = 0;
    *nsol_out = 0;
    if (s1.empty() || s4.empty()) return MSC_NO_REACH;
    // Segment 4 in spatially compact clusters: p3 = t - L4 r_l sorted along a Morton curve
    // and cut into groups of kGmsCluster.  Centres and radii are host estimates; the
    // skip bounds are widened by a margin far above any rounding difference.
    const int n4 = (int)s4.size();
    std::vector<double> P(3 * (size_t)n4);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < n4; ++k)
        for (int d = 0; d < 3; ++d) {
            P[3 * k + d] = a.t[d] - a.L4 * Q[3 * (size_t)s4[k] + d];
            lo[d] = std::min(lo[d], P[3 * k + d]);
            hi[d] = std::max(hi[d], P[3 * k + d]);
        }
    auto morton = [&](int k) {
        uint64_t code = 0;
        for (int d = 0; d < 3; ++d) {
            const double span = hi[d] - lo[d];
            const uint64_t q = span > 0 ? (uint64_t)std::min(1023.0, (P[3 * k + d] - lo[d]) / span * 1023.0) : 0;
            for (int b = 0; b < 10; ++b) code |= ((q >> b) & 1ull) << (3 * b + d);
        }
        return code;
    };
    std::vector<std::pair<uint64_t, int>> mk(n4);
    for (int k = 0; k < n4; ++k) mk[k] = {morton(k), k};
    std::sort(mk.begin(), mk.end());
    std::vector<int32_t> order(n4);
    for (int k = 0; k < n4; ++k) order[k] = s4[mk[k].second];
    const int ncl = (n4 + kGmsCluster - 1) / kGmsCluster;
    std::vector<GmsCluster> cls(ncl);
    const double margin = 1e-6 * (1.0 + a.L3 + a.L4);
    const double rlo = std::sqrt(a.glo), rhi = std::sqrt(a.ghi);
    for (int c0 = 0; c0 < ncl; ++c0) {
        const int b = c0 * kGmsCluster, e = std::min(n4, b + kGmsCluster);
        double ctr[3] = {0, 0, 0};
        for (int k = b; k < e; ++k)
            for (int d = 0; d < 3; ++d) ctr[d] += P[3 * (size_t)mk[k].second + d];
        for (int d = 0; d < 3; ++d) ctr[d] /= (e - b);
        double rad = 0;
        for (int k = b; k < e; ++k) {
            double r2 = 0;
            for (int d = 0; d < 3; ++d) {
                const double u = P[3 * (size_t)mk[k].second + d] - ctr[d];
                r2 += u * u;
            }
            rad = std::max(rad, std::sqrt(r2));
        }
        const double inner = rlo - rad - margin, outer = rhi + rad + margin;
        cls[c0] = GmsCluster{ctr[0], ctr[1], ctr[2], inner > 0 ? inner * inner : -1.0, outer * outer, 0.0};
    }
    void *d_s1, *d_order, *d_pts, *d_cl, *d_per;
    MSC_TRY(arena_alloc(c, s1.size() * 4, &d_s1));
    MSC_TRY(arena_alloc(c, (uint64_t)n4 * 4, &d_order));
    MSC_TRY(arena_alloc(c, (uint64_t)n4 * sizeof(GmsPoint), &d_pts));
    MSC_TRY(arena_alloc(c, (uint64_t)ncl * sizeof(GmsCluster), &d_cl));
    MSC_TRY(arena_alloc(c, s1.size() * 8, &d_per));
    HIP_TRY(hipMemcpyAsync(d_s1, s1.data(), s1.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_order, order.data(), (size_t)n4 * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_cl, cls.data(), (size_t)ncl * sizeof(GmsCluster), hipMemcpyHostToDevice, c->stream));
    LAUNCH(MSC_K_SEED, 1, n4, launch_gms_points(a, (const int32_t*)d_order, n4, (GmsPoint*)d_pts, c->stream));
    const uint64_t cap = std::min<uint64_t>(4ull << 20, free_bytes(c) / 16);
    void* d_keys;
    MSC_TRY(arena_alloc(c, std::max<uint64_t>(cap, 1) * 8, &d_keys));
    LAUNCH(MSC_K_FILL, -1, 0, launch_fill((uint64_t*)c->counters, kCounters, 0ull, c->stream));
    std::vector<unsigned long long> per(s1.size());
    // one pass over the survivors lo..hi: per[] filled, *slots = keys reserved
    auto run = [&](int lo, int hi, uint64_t& slots) -> msc_status {
        unsigned long long* ctr = take_counter(c);
        if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
        LAUNCH(MSC_K_FILL, -1, 0, launch_fill((uint64_t*)d_per, s1.size(), 0ull, c->stream));
        LAUNCH(MSC_K_JOIN, 2, (int64_t)(hi - lo + 1),
               launch_gms_pairs(a, (const int32_t*)d_s1, (int)s1.size(), (const GmsPoint*)d_pts, n4,
                                (const GmsCluster*)d_cl, ncl, ctr, (unsigned long long*)d_per, (uint64_t*)d_keys, cap,
                                lo, hi, 1, c->stream));
        HIP_TRY(hipMemcpyAsync(per.data(), d_per, per.size() * 8, hipMemcpyDeviceToHost, c->stream));
        MSC_TRY(read_counter(c, ctr, &slots));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return MSC_OK;
    };
    // Survivors in chunks (one chunk holding all of them unless first_only; with it, the
    // first chunk covers about 4*2^20 pairs and each next one twice the last).  A chunk's
    // keys are kept when there are few of them; otherwise the chunk's first survivors that,
    // with the earlier chunks, hold the first `want` are searched again and only their
    // keys are kept.
    const int n1 = (int)s1.size();
    int chunk = first_only ? std::max(16, (int)std::min<uint64_t>(n1, (4ull << 20) / (uint64_t)nq)) : n1;
    std::vector<uint64_t> keys;
    uint64_t found = 0;
    for (int lo = 0; lo < n1 && !(first_only && found >= (uint64_t)want); lo += chunk, chunk = std::min(n1, 2 * chunk)) {
        const int hi = std::min(n1, lo + chunk) - 1;
        uint64_t slots = 0;
        MSC_TRY(run(lo, hi, slots));
        uint64_t here = 0;
        for (int ii = lo; ii <= hi; ++ii) here += per[ii];
        uint64_t keep = here;
        if (here > std::min<uint64_t>(cap, kGmsFewKeys)) {
            uint64_t acc = 0;
            int ii0 = lo;
            for (; ii0 <= hi; ++ii0) {
                acc += per[ii0];
                if (found + acc >= (uint64_t)want) break;
            }
            ii0 = std::min(ii0, hi);
            if (acc > cap) return fail(c, MSC_E_CAPACITY, "the first segment-1 vectors hold more than %llu solutions",
                                       (unsigned long long)cap);
            MSC_TRY(run(lo, ii0, slots));
            keep = acc;
        }
        if (slots != keep) return fail(c, MSC_E_STATE, "gap search: %llu keys stored, %llu counted",
                                       (unsigned long long)slots, (unsigned long long)keep);
        const size_t old = keys.size();
        keys.resize(old + keep);
        if (keep) HIP_TRY(hipMemcpyAsync(keys.data() + old, d_keys, keep * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        found += here;
    }
    *count_out = (int64_t)found;
    if (found == 0) return MSC_NO_REACH;
    const int nout = (int)std::min<uint64_t>((uint64_t)want, keys.size());
    std::partial_sort(keys.begin(), keys.begin() + nout, keys.end());
    void *d_sel, *d_vec;
    MSC_TRY(arena_alloc(c, (uint64_t)nout * 8, &d_sel));
    MSC_TRY(arena_alloc(c, (uint64_t)nout * 18 * 8, &d_vec));
    HIP_TRY(hipMemcpyAsync(d_sel, keys.data(), (size_t)nout * 8, hipMemcpyHostToDevice, c->stream));
    LAUNCH(MSC_K_REFINE, -1, nout, launch_gms_vectors(a, (const uint64_t*)d_sel, nout, (double*)d_vec, c->stream));
    HIP_TRY(hipMemcpyAsync(vec_out, d_vec, (size_t)nout * 18 * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < nout; ++k) {
        sols_out[3 * k] = (int32_t)(keys[k] >> 40);
        sols_out[3 * k + 1] = (int32_t)((keys[k] >> 20) & 0xfffff);
        sols_out[3 * k + 2] = (int32_t)(keys[k] & 0xfffff);
    }
    *nsol_out = nout;
    return MSC_OK;
}

// Short-reach path: the reach poses, the shortcut, then the end effector's walk back
// along the shortcut from each reach pose (or, without a hit, the reach-pose-guided walk).
msc_status short_on(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t target[3], int32_t rho2,
                    int32_t K, const msc_track* tr, const msc_opts* opts, int32_t* path_out, int32_t* rows_out,
                    int32_t* hit_out) {
    MSC_TRY(check_scene(c, sc));
    MSC_TRY(check_arm(c, arm, sc->n));
    if (!target || !path_out || !rows_out || !hit_out) return fail(c, MSC_E_ARG, "NULL argument");
    for (int i = 0; i < 3; ++i)
        if (target[i] < 0 || target[i] >= sc->n) return fail(c, MSC_E_ARG, "target outside the grid");
    msc_opts o = opts_or_default(opts);
    if (o.reach_retries < 1 || o.reach_retries > 64 || o.split_m < -1 || o.split_m > arm->dof)
        return fail(c, MSC_E_ARG, "bad options");
    const int n = arm->dof;
    if (K < 2 || K > n - 1) return fail(c, MSC_E_ARG, "shortcut segments outside 2..dof-1");
    if (rho2 < 0 || rho2 > 65535) return fail(c, MSC_E_ARG, "rho2 outside 0..65535");
    TrackArgs ta{};
    MSC_TRY(track_params(c, arm, tr, std::max(1, n - 2), ta));
    const int fallback_tracked = ta.tracked;
    const int max_rows = std::max(arm->samples * (K - 1) + 2, arm->samples * (fallback_tracked - 1) + 1);
    if (max_rows > kTrackMaxPoints) return fail(c, MSC_E_ARG, "more than %d waypoints", kTrackMaxPoints);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    Plan p;
    make_plan(arm, target, p);
    p.prune = (o.flags & MSC_NO_PRUNE) ? 0 : 1;
    p.split = o.split_m;
    // the pruned forward sets keep every hit when rho + 1 <= R_{k+1} for k = 2..K
    int64_t rho = 0;
    while (rho * rho < rho2) ++rho;
    for (int k = 2; k <= K; ++k) {
        TableEntry t;
        MSC_TRY(get_table(c, p.na, p.S, p.len[k], &t));
        if (rho + 1 > isqrt_ceil((int64_t)t.maxn2))
            return fail(c, MSC_E_ARG, "rho + 1 exceeds the reach of segment %d", k + 1);
    }
    for (int i = 0; i < MSC_MAX_DOF + 3; ++i) hit_out[i] = 0;
    ReachOut r;
    msc_status st = run_reach(c, sc, p, o.reach_retries, false, r);
    if (st != MSC_OK) return st;
    const msc_stats keep = c->stats;
    begin_call(c);
    ShortcutHit hit;
    MSC_TRY(shortcut_search(c, sc, p, K, rho2, hit));
    c->stats = keep;
    begin_call(c);
    MSC_TRY(track_arm(c, sc, p, ta));
    if (hit.found) {
        ta.mode = 2;
        ta.tracked = n;
        for (int j = 0; j < hit.k; ++j) ta.guide[j] = hit.q[j];
        ta.guide_k = hit.k;
        ta.guide_s = hit.s;
        hit_out[0] = hit.k;
        hit_out[1] = hit.s;
        hit_out[2] = (int32_t)hit.length;
        for (int j = 0; j < hit.k; ++j) hit_out[3 + j] = hit.q[j] * arm->step_cdeg;
    } else {
        ta.mode = 0;
        ta.tracked = fallback_tracked;
    }
    return track_run(c, ta, r.sols, r.nsol, n, max_rows, arm->step_cdeg, path_out, rows_out);
}

msc_status guided_on(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t target[3], const msc_track* tr,
                     const msc_opts* opts, int32_t* path_out, int32_t* rows_out) {
    if (!path_out || !rows_out) return fail(c, MSC_E_ARG, "NULL output");
    TrackJob job;
    MSC_TRY_STATUS(guided_prepare(c, sc, arm, target, tr, opts, job));
    return track_run(c, job.ta, job.sols, job.nsol, job.width, job.max_rows, job.step, path_out, rows_out);
}

msc_status pose_path_on(Lane* c, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                        const int32_t target[3], const msc_arm* varm, const msc_track* tr, const msc_opts* opts,
                        int32_t* path_out, int32_t* rows_out) {
    if (!path_out || !rows_out) return fail(c, MSC_E_ARG, "NULL output");
    TrackJob job;
    MSC_TRY_STATUS(pose_path_prepare(c, sc, arm, start_cdeg, target, varm, tr, opts, job));
    return track_run(c, job.ta, job.sols, job.nsol, job.width, job.max_rows, job.step, path_out, rows_out);
}

// Tracking launches deferred by a batch with MSC_FUSED_TRACK: all of them in one launch
// on lane c (one block per query), then the rows of each into its query.
msc_status run_fused_tracks(Lane* c, std::vector<std::pair<msc_query*, TrackJob*>>& jobs) {
    constexpr size_t kChunk = 256;   // kernel arguments of a chunk fit the staging buffer
    for (size_t b = 0; b < jobs.size(); b += kChunk) {
        const size_t cnt = std::min(kChunk, jobs.size() - b);
        begin_call(c);
        std::vector<TrackArgs> args(cnt);
        std::vector<void*> h_rows(cnt), h_st(cnt);
        for (size_t j = 0; j < cnt; ++j) {
            TrackJob& job = *jobs[b + j].second;
            void *h_sols, *d_sols, *d_rows, *d_st;
            MSC_TRY(host_area(c, (size_t)job.nsol * job.width * 4, &h_sols, &d_sols));
            MSC_TRY(host_area(c, (size_t)job.max_rows * job.ta.n * 4, &h_rows[j], &d_rows));
            MSC_TRY(host_area(c, 16, &h_st[j], &d_st));
            std::memcpy(h_sols, job.sols.data(), (size_t)job.nsol * job.width * 4);
            args[j] = job.ta;
            args[j].nsol = job.nsol;
            args[j].sols = (const int32_t*)d_sols;
            args[j].rows = (int32_t*)d_rows;
            args[j].status = (int32_t*)d_st;
        }
        void* d_args;
        MSC_TRY(upload(c, args.data(), cnt * sizeof(TrackArgs), &d_args));
        LAUNCH(MSC_K_TRACK, -1, (int64_t)cnt, launch_track_batch((const TrackArgs*)d_args, (int)cnt, c->stream));
        MSC_TRY(sync_lane(c));
        for (size_t j = 0; j < cnt; ++j) {
            msc_query* q = jobs[b + j].first;
            TrackJob& job = *jobs[b + j].second;
            const volatile int32_t* st = (const volatile int32_t*)h_st[j];
            const int rows = st[0];
            if (rows <= 0) {
                q->status = MSC_NO_PATH;
                continue;
            }
            if (rows > job.max_rows) {
                q->status = MSC_E_CAPACITY;
                std::snprintf(q->error, sizeof q->error, "tracked path longer than planned");
                continue;
            }
            const int32_t* hr = (const int32_t*)h_rows[j];
            for (size_t i = 0; i < (size_t)rows * job.ta.n; ++i) q->out[i] = hr[i] * job.step;
            q->rows = rows;
            q->status = MSC_OK;
        }
    }
    return MSC_OK;
}

// Solves q on lane L against the grid held by binding b, writes q->status, q->tick and
// q->error, and releases the binding.
// deferred: a kind 2 / 3 query of a fused batch leaves its tracking in *deferred (and
// keeps the binding) instead of running it; returns true when it did.
bool query_on(Lane* L, msc_query* q, const msc_opts* opts, Binding& b, TrackJob* deferred = nullptr) {
    msc_status st;
    L->err.clear();
    q->rows = 0;
    if (!q->scene || !q->arm || !q->out) {
        st = fail(L, MSC_E_ARG, "query with a NULL scene, arm or output");
    } else {
        prof_reset(L, opts ? opts->flags : 0u);
        if (b.ready && L->stream != L->owner->stream) (void)hipStreamWaitEvent(L->stream, b.ready, 0);
        const msc_scene* sc = &b.view;
        if (q->kind == 0) {
            st = reach_on(L, sc, q->arm, q->target, opts, q->out);
        } else if (q->kind == 1) {
            st = path_on(L, sc, q->arm, q->start_cdeg, q->target, q->waypoints, q->max_delta_cdeg, opts, q->out,
                         q->ref_cdeg);
        } else if (q->kind == 2 || q->kind == 3) {
            TrackJob own;
            TrackJob& job = deferred ? *deferred : own;
            st = q->kind == 2 ? guided_prepare(L, sc, q->arm, q->target, &q->track, opts, job)
                              : pose_path_prepare(L, sc, q->arm, q->start_cdeg, q->target, q->virtual_arm, &q->track,
                                                  opts, job);
            if (st == MSC_OK && deferred) {
                prof_finish(L);
                return true;
            }
            if (st == MSC_OK)
                st = track_run(L, job.ta, job.sols, job.nsol, job.width, job.max_rows, job.step, q->out, &q->rows);
        } else {
            st = fail(L, MSC_E_ARG, "query kind %d", q->kind);
        }
        prof_finish(L);
    }
    // a call that failed part-way may leave kernels in flight that read the grid
    if (st < 0) (void)hipStreamSynchronize(L->stream);
    q->status = st;
    q->tick = b.view.tick;
    std::snprintf(q->error, sizeof q->error, "%s", st < 0 ? L->err.c_str() : "");
    unbind_scene(b);
    return false;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// Server state: a queue of submitted queries served by one host thread per worker
// lane, the server's logical clock and the paths executing on it ("Dynamic
// Obstacles": an arm in motion along a computed path, replanned midcourse when a
// moving obstacle will block a waypoint ahead of it).
// ---------------------------------------------------------------------------
namespace {

// A path executing on the logical clock: waypoint w is reached at start_tick + w * tpw.
struct Exec {
    const msc_scene* scene = nullptr;
    msc_arm arm{};
    std::vector<int32_t> rows;   // (W + 1) * dof centidegrees
    int W = 0;
    int32_t target[3] = {0, 0, 0};
    int32_t max_delta_cdeg = 0;
    int64_t start_tick = 0;
    int32_t tpw = 0;
    int32_t depth = 0;           // replans that led to this path
};

// A replan issued by msc_server_step: its query record and the arrays it points to.
struct ReplanRec {
    msc_query q{};
    msc_arm arm{};
    std::vector<int32_t> start, ref, out;
    double issued_ms = 0.0;
};

struct Job {
    uint64_t ticket = 0;
    msc_query* q = nullptr;
    Binding bind;
    ReplanRec* rec = nullptr;    // set for a replan issued by the server
};

}  // namespace

struct ServerState {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job> queue;
    size_t max_pending = 0;                  // submissions refused while this many wait (0: no limit)
    std::map<uint64_t, double> submitted;   // ticket -> submission time (ms), until finished
    std::set<uint64_t> done;                 // finished, not yet reported by poll / wait
    std::condition_variable done_cv;
    std::vector<std::thread> threads;
    msc_opts opts{};
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t tick = 0;
    std::vector<Exec> executing;
    std::map<uint64_t, std::unique_ptr<ReplanRec>> replans;   // issued replans, by ticket
    std::vector<uint64_t> replans_done;                        // finished, not yet taken
    std::vector<std::unique_ptr<ReplanRec>> taken;             // returned by the last take
};

namespace {

// Validity of the remaining waypoints of executing paths on the grids of the current
// tick: one pose-check launch per (path), reading its rows from the control lane's
// mapped staging memory and writing its verdicts there; the launches of as many paths
// as fit the staging buffer run back to back, then one wait.
msc_status revalidate(Lane* c, const std::vector<Exec>& ex, const std::vector<std::pair<size_t, int>>& live,
                      std::vector<std::vector<uint8_t>>& valid) {
    valid.assign(live.size(), {});
    struct Pending {
        size_t item;
        uint8_t* host;
        int rows;
    };
    std::vector<Pending> pend;
    begin_call(c);
    auto flush = [&]() -> msc_status {
        if (pend.empty()) return MSC_OK;
        MSC_TRY(sync_lane(c));
        for (const Pending& p : pend) valid[p.item].assign(p.host, p.host + p.rows);
        pend.clear();
        begin_call(c);
        return MSC_OK;
    };
    for (size_t i = 0; i < live.size(); ++i) {
        const Exec& e = ex[live[i].first];
        const int d = live[i].second;
        const int n = e.arm.dof;
        const int rows = e.W - d + 1;
        const size_t qbytes = (size_t)rows * n * 4;
        if (qbytes + (size_t)rows + 1024 > kStagingBytes / 2)
            return fail(c, MSC_E_CAPACITY, "executing path of %d waypoints too long to re-validate", e.W);
        if (c->staging_used + qbytes + (size_t)rows + 1024 > kStagingBytes - 4096) MSC_TRY(flush());
        Plan p;
        make_plan(&e.arm, nullptr, p);
        std::vector<JointView> jv;
        MSC_TRY(joint_views(c, p, jv));
        void *hq, *dq, *hv, *dv;
        MSC_TRY(host_area(c, qbytes, &hq, &dq));
        MSC_TRY(host_area(c, (size_t)rows, &hv, &dv));
        int32_t* qs = (int32_t*)hq;
        for (size_t j = 0; j < (size_t)rows * n; ++j) qs[j] = e.rows[(size_t)d * n + j] / e.arm.step_cdeg;
        PoseArgs a{};
        for (int k = 0; k < n; ++k) a.joints[k] = jv[k];
        a.g = grid_view(e.scene);
        a.n = n;
        a.na = p.na;
        a.bx = p.base[0];
        a.by = p.base[1];
        a.bz = p.base[2];
        a.ia0 = p.ia0;
        a.ie0 = p.ie0;
        LAUNCH(MSC_K_POSE, -1, rows, launch_pose_check(a, (const int32_t*)dq, rows, (uint8_t*)dv, nullptr, c->stream));
        pend.push_back({i, (uint8_t*)hv, rows});
    }
    return flush();
}

}  // namespace

extern "C" {

void msc_opts_default(msc_opts* o) {
    if (!o) return;
    o->split_m = -1;
    o->tube_r0 = 1;
    o->tube_r1 = 2;
    o->reach_retries = 4;
    o->flags = 0;
    o->approach_az_cdeg = 0;
    o->approach_el_cdeg = 0;
    o->approach_half_cdeg = -1;
}

msc_status msc_ctx_create(int device, void* hip_stream, void* dev_workspace, uint64_t ws_bytes, msc_ctx** out) {
    if (!out || !dev_workspace) return MSC_E_ARG;
    if (ws_bytes < (64ull << 20)) return MSC_E_ARG;
    if ((uintptr_t)dev_workspace % kAlign) return MSC_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return MSC_E_HIP;
    if (static_scratch_init(device) != hipSuccess) return MSC_E_HIP;
    msc_ctx* o = new (std::nothrow) msc_ctx();
    if (!o) return MSC_E_NOMEM;
    o->device = device;
    o->stream = (hipStream_t)hip_stream;
    o->ws = (char*)dev_workspace;
    o->ws_bytes = ws_bytes;
    uint64_t table_bytes = std::min<uint64_t>(256ull << 20, ws_bytes / 8) & ~(kAlign - 1);
    o->table_lo = ws_bytes - table_bytes;
    o->table_top = ws_bytes & ~(kAlign - 1);   // keeps table rows aligned
    msc_status st = layout_lanes(o, 0);
    if (st != MSC_OK) {
        lane_free(o->control);
        delete o;
        return st;
    }
    // a tuning cache named by the environment, when it exists and fits this GPU
    const char* cache = std::getenv("MSC_TUNE_CACHE");
    if (cache && *cache) {
        if (FILE* f = std::fopen(cache, "r")) {
            std::fclose(f);
            (void)msc_tune_load(o, cache);
            o->err.clear();
        }
    }
    *out = o;
    return MSC_OK;
}

msc_status msc_ctx_destroy(msc_ctx* o) {
    if (!o) return MSC_E_ARG;
    (void)hipSetDevice(o->device);
    if (o->server) msc_server_stop(o);
    for (Lane* w : o->workers) lane_free(w);
    lane_free(o->control);
    delete o;
    return MSC_OK;
}

msc_status msc_ctx_set_lanes(msc_ctx* o, int32_t nworkers) {
    if (!o) return MSC_E_ARG;
    if (nworkers < 0 || nworkers > 64) return ctx_fail(o, MSC_E_ARG, "nworkers outside 0..64");
    if (o->server) return ctx_fail(o, MSC_E_STATE, "the server is running");
    if (hipSetDevice(o->device) != hipSuccess) return MSC_E_HIP;
    (void)hipStreamSynchronize(o->stream);
    return layout_lanes(o, nworkers);
}

uint64_t msc_lane_bytes(msc_ctx* o) { return (o && o->control) ? o->control->hi : 0; }

uint64_t msc_scene_bytes(int32_t n) {
    if (n <= 0) return 0;
    uint64_t wpr = ((uint64_t)n + 63) / 64;
    return (uint64_t)n * n * wpr * 8;
}

msc_status msc_scene_create(msc_ctx* o, int32_t n, int32_t dilate_r, const msc_box* boxes, int32_t nbox,
                            const msc_sphere* spheres, int32_t nsph, void* dev_grid, uint64_t grid_bytes,
                            msc_scene** out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;

    if (!out || !dev_grid) return fail(c, MSC_E_ARG, "NULL output or grid buffer");
    if (n < 1 || n > 1024) return fail(c, MSC_E_ARG, "grid size %d outside 1..1024", n);
    if (dilate_r < 0 || nbox < 0 || nsph < 0) return fail(c, MSC_E_ARG, "negative dilation or count");
    if ((nbox && !boxes) || (nsph && !spheres)) return fail(c, MSC_E_ARG, "NULL obstacle array");
    for (int i = 0; i < nbox; ++i)
        for (int a = 0; a < 3; ++a)
            if (boxes[i].ext[a] < 1) return fail(c, MSC_E_ARG, "box %d has an extent < 1", i);
    for (int i = 0; i < nsph; ++i)
        if (spheres[i].r < 0) return fail(c, MSC_E_ARG, "sphere %d has a negative radius", i);
    if (grid_bytes < msc_scene_bytes(n)) return fail(c, MSC_E_NOMEM, "grid buffer too small");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    msc_scene* s = new (std::nothrow) msc_scene();
    if (!s) return fail(c, MSC_E_NOMEM, "host allocation");
    s->ctx = c->owner;
    s->n = n;
    s->wpr = (n + 63) / 64;
    s->dilate = dilate_r;
    s->grid = (uint64_t*)dev_grid;
    s->bytes = grid_bytes;
    hipError_t e = hipSuccess;
    if ((int64_t)nbox * 6 + (int64_t)nsph * 4 <= kRasterInline) {
        // the obstacle lists travel in the kernel's arguments: nothing on the host has to
        // outlive the launch, so the call does not wait for the raster
        RasterInline inl{};
        for (int i = 0; i < nbox; ++i)
            for (int a = 0; a < 3; ++a) {
                inl.v[i * 6 + a] = boxes[i].lo[a];
                inl.v[i * 6 + 3 + a] = boxes[i].ext[a];
            }
        for (int i = 0; i < nsph; ++i) {
            for (int a = 0; a < 3; ++a) inl.v[nbox * 6 + i * 4 + a] = spheres[i].c[a];
            inl.v[nbox * 6 + i * 4 + 3] = spheres[i].r;
        }
        e = launch_raster_inline(s->grid, n, s->wpr, dilate_r, inl, nbox, nsph, c->stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(s->ready, c->stream);
    } else {
        std::vector<int32_t> hb((size_t)std::max(nbox, 1) * 6), hs((size_t)std::max(nsph, 1) * 4);
        for (int i = 0; i < nbox; ++i)
            for (int a = 0; a < 3; ++a) {
                hb[i * 6 + a] = boxes[i].lo[a];
                hb[i * 6 + 3 + a] = boxes[i].ext[a];
            }
        for (int i = 0; i < nsph; ++i) {
            for (int a = 0; a < 3; ++a) hs[i * 4 + a] = spheres[i].c[a];
            hs[i * 4 + 3] = spheres[i].r;
        }
        // long lists: read from mapped host memory when they fit the staging buffer, else
        // from a device copy; the call waits for the raster before the staging is reused
        void *hbp, *db, *hsp, *ds;
        const size_t obytes = (hb.size() + hs.size()) * 4;
        msc_status st = MSC_OK;
        if (obytes + 1024 <= kStagingBytes / 2) {
            st = host_area(c, hb.size() * 4, &hbp, &db);
            if (st == MSC_OK) st = host_area(c, hs.size() * 4, &hsp, &ds);
            if (st == MSC_OK) {
                std::memcpy(hbp, hb.data(), hb.size() * 4);
                std::memcpy(hsp, hs.data(), hs.size() * 4);
            }
        } else {
            st = arena_alloc(c, hb.size() * 4, &db);
            if (st == MSC_OK) st = arena_alloc(c, hs.size() * 4, &ds);
            if (st == MSC_OK) e = hipMemcpyAsync(db, hb.data(), hb.size() * 4, hipMemcpyHostToDevice, c->stream);
            if (st == MSC_OK && e == hipSuccess)
                e = hipMemcpyAsync(ds, hs.data(), hs.size() * 4, hipMemcpyHostToDevice, c->stream);
        }
        if (st != MSC_OK) {
            delete s;
            return st;
        }
        if (e == hipSuccess)
            e = launch_raster(s->grid, n, s->wpr, dilate_r, (const int32_t*)db, nbox, (const int32_t*)ds, nsph,
                              c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) {
        if (s->ready) (void)hipEventDestroy(s->ready);
        delete s;
        return fail(c, MSC_E_HIP, "raster: %s", hipGetErrorString(e));
    }
    // room for grids of ticks: slot 0 keeps the static grid, the others take
    // msc_scene_set_dynamic
    const uint64_t one = msc_scene_bytes(n);
    const uint64_t slots = std::min<uint64_t>(grid_bytes / one, (uint64_t)kMaxTickGrids + 1);
    if (slots >= 2) {
        s->dyn = new (std::nothrow) SceneDyn();
        if (!s->dyn) {
            msc_scene_destroy(s);
            return fail(c, MSC_E_NOMEM, "host allocation");
        }
        s->dyn->slot.resize(slots);
        for (uint64_t i = 0; i < slots; ++i) {
            GridSlot& g = s->dyn->slot[i];
            g.grid = (uint64_t*)((char*)dev_grid + i * one);
            if (i > 0 && hipEventCreateWithFlags(&g.ready, hipEventDisableTiming) != hipSuccess) {
                msc_scene_destroy(s);
                return fail(c, MSC_E_HIP, "hipEventCreateWithFlags");
            }
        }
        s->dyn->cur = 0;
    }
    *out = s;
    return MSC_OK;
}

msc_status msc_scene_destroy(msc_scene* s) {
    if (!s) return MSC_E_ARG;
    if (s->ready) (void)hipEventDestroy(s->ready);
    if (s->dyn) {
        for (GridSlot& g : s->dyn->slot)
            if (g.ready) (void)hipEventDestroy(g.ready);
        delete s->dyn;
    }
    delete s;
    return MSC_OK;
}

uint64_t msc_scene_bytes_dynamic(int32_t n, int32_t ticks) {
    if (n <= 0 || ticks < 1 || ticks > kMaxTickGrids) return 0;
    return msc_scene_bytes(n) * (uint64_t)(ticks + 1);
}

msc_status msc_scene_set_dynamic(msc_scene* s, const msc_box* boxes, int32_t nbox, int64_t tick) {
    if (!s) return MSC_E_ARG;
    msc_ctx* o = s->ctx;
    Lane* c = o->control;
    if (nbox < 0 || (nbox && !boxes)) return fail(c, MSC_E_ARG, "bad moving-box array");
    for (int i = 0; i < nbox; ++i)
        for (int a = 0; a < 3; ++a)
            if (boxes[i].ext[a] < 1) return fail(c, MSC_E_ARG, "moving box %d has an extent < 1", i);
    if (!s->dyn) return fail(c, MSC_E_NOMEM, "the scene buffer holds no grids of ticks (msc_scene_bytes_dynamic)");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    SceneDyn* d = s->dyn;
    std::lock_guard<std::mutex> lock(d->mu);
    // the oldest slot no query uses; the current one only when it is the last free one
    // (calls that read it without a binding run on this stream and have returned)
    int pick = -1;
    for (int i = 1; i < (int)d->slot.size(); ++i) {
        if (i == d->cur || d->slot[i].refs > 0) continue;
        if (pick < 0 || d->slot[i].tick < d->slot[pick].tick) pick = i;
    }
    if (pick < 0 && d->cur > 0 && d->slot[d->cur].refs == 0) pick = d->cur;
    if (pick < 0) return fail(c, MSC_E_CAPACITY, "every grid of a tick is in use by queries");
    GridSlot& g = d->slot[pick];
    const uint64_t* src = d->slot[0].grid;
    for (int b0 = 0; b0 == 0 || b0 < nbox; b0 += kDynBoxes) {
        DynBoxes db{};
        db.count = std::min(kDynBoxes, nbox - b0);
        for (int i = 0; i < db.count; ++i)
            for (int a = 0; a < 3; ++a) {
                db.b[i * 6 + a] = boxes[b0 + i].lo[a];
                db.b[i * 6 + 3 + a] = boxes[b0 + i].ext[a];
            }
        HIP_TRY(launch_raster_dyn(g.grid, src, s->n, s->wpr, s->dilate, db, c->stream));
        src = g.grid;
    }
    HIP_TRY(hipEventRecord(g.ready, c->stream));
    g.tick = tick;
    d->cur = pick;
    s->grid = g.grid;
    s->tick = tick;
    return MSC_OK;
}

msc_status msc_reach(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t target[3],
                     const msc_opts* opts, int32_t* angles_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, opts ? opts->flags : 0u);
    msc_status st = reach_on(c, sc, arm, target, opts, angles_out);
    prof_finish(c);
    return st;
}

msc_status msc_path(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                    const int32_t target[3], int32_t waypoints, int32_t max_delta_cdeg, const msc_opts* opts,
                    int32_t* path_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, opts ? opts->flags : 0u);
    msc_status st = path_on(c, sc, arm, start_cdeg, target, waypoints, max_delta_cdeg, opts, path_out);
    prof_finish(c);
    return st;
}

msc_status msc_replan(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                      const int32_t target[3], int32_t waypoints, int32_t max_delta_cdeg, const int32_t* ref_cdeg,
                      const msc_opts* opts, int32_t* path_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    if (!ref_cdeg) return fail(c, MSC_E_ARG, "NULL reference path");
    prof_reset(c, opts ? opts->flags : 0u);
    msc_status st = path_on(c, sc, arm, start_cdeg, target, waypoints, max_delta_cdeg, opts, path_out, ref_cdeg);
    prof_finish(c);
    return st;
}

void msc_track_default(msc_track* t) {
    if (!t) return;
    t->tracked = -1;
    t->max_delta_cdeg = -1;
    t->relaxed_delta_cdeg = -1;
    t->eps2_vox = 9;
}

msc_status msc_guided_path(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t target[3],
                           const msc_track* track, const msc_opts* opts, int32_t* path_out, int32_t* rows_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, opts ? opts->flags : 0u);
    msc_status st = guided_on(c, sc, arm, target, track, opts, path_out, rows_out);
    prof_finish(c);
    return st;
}

msc_status msc_short_path(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t target[3],
                          int32_t rho2_vox, int32_t segments, const msc_track* track, const msc_opts* opts,
                          int32_t* path_out, int32_t* rows_out, int32_t* hit_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, opts ? opts->flags : 0u);
    msc_status st = short_on(c, sc, arm, target, rho2_vox, segments, track, opts, path_out, rows_out, hit_out);
    prof_finish(c);
    return st;
}

int32_t msc_gms_quiver(int32_t step_cdeg, int32_t min_ring, double* out, int32_t cap) {
    std::vector<double> Q;
    if (!build_quiver(step_cdeg, min_ring, Q)) return 0;
    const int32_t n = (int32_t)(Q.size() / 3);
    if (out && cap > 0) std::memcpy(out, Q.data(), (size_t)std::min(n, cap) * 3 * sizeof(double));
    return n;
}

msc_status msc_gms_reach(msc_ctx* o, const msc_scene* sc, const msc_gms_arm* arm, const int32_t target[3],
                         int32_t want, int64_t* count_out, int32_t* sols_out, double* vec_out, int32_t* nsol_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, 0u);
    msc_status st = gms_on(c, sc, arm, target, want, false, count_out, sols_out, vec_out, nsol_out);
    prof_finish(c);
    return st;
}

msc_status msc_gms_reach_first(msc_ctx* o, const msc_scene* sc, const msc_gms_arm* arm, const int32_t target[3],
                               int32_t want, int64_t* count_out, int32_t* sols_out, double* vec_out,
                               int32_t* nsol_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, 0u);
    msc_status st = gms_on(c, sc, arm, target, want, true, count_out, sols_out, vec_out, nsol_out);
    prof_finish(c);
    return st;
}

msc_status msc_pose_path(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                         const int32_t target[3], const msc_arm* virtual_arm, const msc_track* track,
                         const msc_opts* opts, int32_t* path_out, int32_t* rows_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;
    prof_reset(c, opts ? opts->flags : 0u);
    msc_status st = pose_path_on(c, sc, arm, start_cdeg, target, virtual_arm, track, opts, path_out, rows_out);
    prof_finish(c);
    return st;
}

msc_status msc_get_timings(msc_ctx* o, msc_timing* out, int32_t cap, int32_t* count) {
    if (!o || !count || cap < 0 || (cap && !out)) return MSC_E_ARG;
    Lane* c = o->control;
    *count = (int32_t)c->recs.size();
    for (int32_t i = 0; i < cap && i < (int32_t)c->recs.size(); ++i) out[i] = c->recs[i];
    return MSC_OK;
}

msc_status msc_batch(msc_ctx* o, msc_query* q, int32_t nq, const msc_opts* opts) {
    if (!o) return MSC_E_ARG;
    if (nq < 0 || (nq && !q)) return ctx_fail(o, MSC_E_ARG, "bad query array");
    if (o->server) return ctx_fail(o, MSC_E_STATE, "the server is running");
    const double t0 = now_ms();
    const bool fused = opts && (opts->flags & MSC_FUSED_TRACK);
    std::vector<TrackJob> jobs(fused ? (size_t)nq : 0);
    std::vector<Binding> held(fused ? (size_t)nq : 0);
    std::vector<char> deferred(fused ? (size_t)nq : 0, 0);
    auto one = [&](Lane* L, int32_t i) {
        Binding b = bind_scene(q[i].scene);
        const bool defer = fused && (q[i].kind == 2 || q[i].kind == 3);
        if (query_on(L, &q[i], opts, b, defer ? &jobs[i] : nullptr)) {
            held[i] = b;   // the grid stays bound until the fused launch has run
            deferred[i] = 1;
            return;
        }
        q[i].latency_ms = (float)(now_ms() - t0);
    };
    if (o->workers.empty()) {
        for (int32_t i = 0; i < nq; ++i) one(o->control, i);
    } else {
        std::atomic<int32_t> next{0};
        std::vector<std::thread> threads;
        for (Lane* L : o->workers) {
            threads.emplace_back([&, L]() {
                (void)hipSetDevice(o->device);
                for (int32_t i = next.fetch_add(1); i < nq; i = next.fetch_add(1)) one(L, i);
            });
        }
        for (auto& t : threads) t.join();
    }
    if (!fused) return MSC_OK;
    std::vector<std::pair<msc_query*, TrackJob*>> pending;
    for (int32_t i = 0; i < nq; ++i)
        if (deferred[i]) pending.emplace_back(&q[i], &jobs[i]);
    if (pending.empty()) return MSC_OK;
    Lane* c = o->control;
    prof_reset(c, opts->flags);
    // the searches ran on the worker streams: their grids and tables are complete once
    // those streams are idle
    for (Lane* L : o->workers) (void)hipStreamSynchronize(L->stream);
    c->err.clear();
    msc_status st = run_fused_tracks(c, pending);
    prof_finish(c);
    const double t1 = now_ms();
    for (int32_t i = 0; i < nq; ++i) {
        if (!deferred[i]) continue;
        if (st != MSC_OK) {
            q[i].status = st;
            std::snprintf(q[i].error, sizeof q[i].error, "%s", c->err.c_str());
        }
        q[i].latency_ms = (float)(t1 - t0);
        unbind_scene(held[i]);
    }
    return MSC_OK;
}

msc_status msc_autotune(msc_ctx* o, msc_query* q, int32_t nq, const msc_opts* opts, const char* cache_path) {
    if (!o) return MSC_E_ARG;
    if (nq <= 0 || !q) return ctx_fail(o, MSC_E_ARG, "no queries to tune on");
    if (o->server) return ctx_fail(o, MSC_E_STATE, "the server is running");
    Lane* c = o->control;
    msc_opts po = opts_or_default(opts);
    po.flags = (po.flags | MSC_PROFILE) & ~(MSC_CAPTURE_SETS | MSC_FUSED_TRACK);
    const size_t cells = (size_t)MSC_K_COUNT * 64;
    std::vector<double> sum(cells * kNumShapes, 0.0);
    std::vector<int> cnt(cells * kNumShapes, 0);
    constexpr int kReps = 3;   // the first solve of each variant warms up
    for (int v = 0; v < kNumShapes; ++v) {
        o->tune_force = v;
        for (int rep = 0; rep < kReps; ++rep) {
            for (int32_t i = 0; i < nq; ++i) {
                Binding b = bind_scene(q[i].scene);
                query_on(c, &q[i], &po, b);
                if (q[i].status < 0) {
                    o->tune_force = -1;
                    o->err = q[i].error;
                    return q[i].status;
                }
                if (rep == 0) continue;
                for (const msc_timing& r : c->recs) {
                    if (!tunable(r.kernel) || r.ms < 0) continue;
                    const size_t cell = (size_t)r.kernel * 64 + size_class((uint64_t)std::max<int64_t>(r.in_count, 0));
                    sum[cell * kNumShapes + v] += r.ms;
                    cnt[cell * kNumShapes + v] += 1;
                }
            }
        }
    }
    o->tune_force = -1;
    std::memset(o->tune, -1, sizeof o->tune);
    for (size_t cell = 0; cell < cells; ++cell) {
        const int n0 = cnt[cell * kNumShapes];
        if (n0 == 0) continue;
        int best = 0;
        bool same = true;
        for (int v = 1; v < kNumShapes; ++v) {
            same = same && cnt[cell * kNumShapes + v] == n0;
            if (sum[cell * kNumShapes + v] < sum[cell * kNumShapes + best]) best = v;
        }
        if (same) o->tune[cell / 64][cell % 64] = (int8_t)best;
    }
    if (!cache_path) return MSC_OK;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o->device) != hipSuccess) return ctx_fail(o, MSC_E_HIP, "device properties");
    FILE* f = std::fopen(cache_path, "w");
    if (!f) return ctx_fail(o, MSC_E_ARG, "cannot write the tuning cache");
    std::fprintf(f, "msc-tune 1\ndevice %s\n", prop.gcnArchName);
    for (int k = 0; k < MSC_K_COUNT; ++k)
        for (int cl = 0; cl < 64; ++cl)
            if (o->tune[k][cl] >= 0) {
                const Shape& sh = kShapes[o->tune[k][cl]];
                std::fprintf(f, "entry %d %d %d %u %d\n", k, cl, (int)o->tune[k][cl], sh.max_blocks, sh.lg_bias);
            }
    const bool ok = std::fclose(f) == 0;
    return ok ? MSC_OK : ctx_fail(o, MSC_E_ARG, "cannot write the tuning cache");
}

msc_status msc_tune_load(msc_ctx* o, const char* cache_path) {
    if (!o || !cache_path) return MSC_E_ARG;
    if (o->server) return ctx_fail(o, MSC_E_STATE, "the server is running");
    FILE* f = std::fopen(cache_path, "r");
    if (!f) return ctx_fail(o, MSC_E_ARG, "cannot read the tuning cache");
    char line[512];
    int8_t tune[MSC_K_COUNT][64];
    std::memset(tune, -1, sizeof tune);
    msc_status st = MSC_OK;
    int lineno = 0;
    bool device_ok = false;
    hipDeviceProp_t prop;
    const bool have_prop = hipGetDeviceProperties(&prop, o->device) == hipSuccess;
    while (st == MSC_OK && std::fgets(line, sizeof line, f)) {
        ++lineno;
        char dev[256];
        int k, cl, v, bias;
        unsigned mb;
        if (lineno == 1) {
            if (std::strncmp(line, "msc-tune 1", 10) != 0) st = ctx_fail(o, MSC_E_ARG, "not a tuning cache");
        } else if (lineno == 2) {
            if (std::sscanf(line, "device %255s", dev) != 1) {
                st = ctx_fail(o, MSC_E_ARG, "tuning cache without a device line");
            } else {
                device_ok = have_prop && std::strcmp(dev, prop.gcnArchName) == 0;
                if (!device_ok) st = ctx_fail(o, MSC_E_STATE, "tuning cache of another GPU model");
            }
        } else if (std::sscanf(line, "entry %d %d %d %u %d", &k, &cl, &v, &mb, &bias) == 5) {
            if (k < 0 || k >= MSC_K_COUNT || !tunable(k) || cl < 0 || cl >= 64 || v < 0 || v >= kNumShapes ||
                kShapes[v].max_blocks != mb || kShapes[v].lg_bias != bias)
                st = ctx_fail(o, MSC_E_ARG, "tuning cache entry this library does not have");
            else
                tune[k][cl] = (int8_t)v;
        } else {
            st = ctx_fail(o, MSC_E_ARG, "malformed tuning cache line");
        }
    }
    std::fclose(f);
    if (st == MSC_OK && !device_ok) st = ctx_fail(o, MSC_E_ARG, "tuning cache without a device line");
    if (st == MSC_OK) std::memcpy(o->tune, tune, sizeof tune);
    return st;
}

msc_status msc_tune_entries(msc_ctx* o, int32_t* out, int32_t cap, int32_t* count) {
    if (!o || !count || cap < 0 || (cap && !out)) return MSC_E_ARG;
    int32_t n = 0;
    for (int k = 0; k < MSC_K_COUNT; ++k)
        for (int cl = 0; cl < 64; ++cl)
            if (o->tune[k][cl] >= 0) {
                if (n < cap) {
                    const int v = o->tune[k][cl];
                    out[5 * n] = k;
                    out[5 * n + 1] = cl;
                    out[5 * n + 2] = v;
                    out[5 * n + 3] = (int32_t)kShapes[v].max_blocks;
                    out[5 * n + 4] = kShapes[v].lg_bias;
                }
                ++n;
            }
    *count = n;
    return MSC_OK;
}

uint64_t msc_query_bytes(const msc_query* q) {
    if (!q || !q->arm || !q->scene) return 0;
    // two dense stage sets over a middle-stage pruning box, the tube arrays at radius 2,
    // lists and tables
    const msc_arm* a = q->arm;
    const int n = a->dof;
    if (a->step_cdeg <= 0) return 0;
    const uint64_t na = 36000 / (uint64_t)a->step_cdeg;
    // the pathways meet late (the backward side starts from every orientation), about
    // 5/8 of the way: the dense sets cover a box of the remaining segments' reach
    int64_t reach = 0;
    for (int k = (5 * n + 7) / 8; k < n; ++k) reach += a->len_vox[k] + 1;
    uint64_t edge = std::min<uint64_t>(2 * (uint64_t)reach + 1, (uint64_t)q->scene->n);
    uint64_t dense = edge * edge * edge * na * na / 8;
    uint64_t tube = 0;
    if (q->kind == 1) {
        uint64_t slab = 1;
        for (int k = 0; k < n && slab < (1ull << 40); ++k) slab *= 5;
        tube = 2 * slab * (uint64_t)(q->waypoints + 1);
    }
    return 3 * dense + tube + (64ull << 20);
}

static void server_worker(msc_ctx* o, Lane* L) {
    (void)hipSetDevice(o->device);
    ServerState* S = o->server;
    while (true) {
        Job job;
        {
            std::unique_lock<std::mutex> lock(S->mu);
            S->cv.wait(lock, [&] { return S->stop || !S->queue.empty(); });
            if (S->queue.empty()) return;  // stop requested and nothing left
            job = std::move(S->queue.front());
            S->queue.pop_front();
        }
        msc_query* q = job.q;
        query_on(L, q, &S->opts, job.bind);
        const double t = now_ms();
        {
            std::lock_guard<std::mutex> lock(S->mu);
            if (job.rec) {
                q->latency_ms = (float)(t - job.rec->issued_ms);
                S->replans_done.push_back(job.ticket);
            } else {
                q->latency_ms = (float)(t - S->submitted[job.ticket]);
            }
            // a solved path that is to be executed starts at the current tick
            if (q->kind == 1 && q->execute_ticks > 0 && q->status == MSC_OK) {
                Exec e;
                e.scene = q->scene;
                e.arm = *q->arm;
                e.W = q->waypoints;
                e.rows.assign(q->out, q->out + (size_t)(q->waypoints + 1) * q->arm->dof);
                for (int i = 0; i < 3; ++i) e.target[i] = q->target[i];
                e.max_delta_cdeg = q->max_delta_cdeg;
                e.start_tick = S->tick;
                e.tpw = q->execute_ticks;
                e.depth = q->replan_depth;
                S->executing.push_back(std::move(e));
            }
            if (!job.rec) {
                S->submitted.erase(job.ticket);
                S->done.insert(job.ticket);
            }
        }
        S->done_cv.notify_all();
    }
}

msc_status msc_server_start(msc_ctx* o, const msc_opts* opts) {
    if (!o) return MSC_E_ARG;
    if (o->server) return ctx_fail(o, MSC_E_STATE, "the server is already running");
    if (o->workers.empty()) return ctx_fail(o, MSC_E_STATE, "no worker lanes (msc_ctx_set_lanes)");
    ServerState* S = new (std::nothrow) ServerState();
    if (!S) return MSC_E_NOMEM;
    msc_opts_default(&S->opts);
    if (opts) S->opts = *opts;
    o->server = S;
    for (Lane* L : o->workers) S->threads.emplace_back(server_worker, o, L);
    return MSC_OK;
}

msc_status msc_server_set_limit(msc_ctx* o, int32_t max_pending) {
    if (!o) return MSC_E_ARG;
    if (max_pending < 0) return ctx_fail(o, MSC_E_ARG, "max_pending < 0");
    ServerState* S = o->server;
    if (!S) return ctx_fail(o, MSC_E_STATE, "the server is not running");
    std::lock_guard<std::mutex> lock(S->mu);
    S->max_pending = (size_t)max_pending;
    return MSC_OK;
}

msc_status msc_server_submit(msc_ctx* o, msc_query* q, uint64_t* ticket) {
    if (!o || !q || !ticket) return MSC_E_ARG;
    ServerState* S = o->server;
    if (!S) return ctx_fail(o, MSC_E_STATE, "the server is not running");
    if (q->execute_ticks < 0) return ctx_fail(o, MSC_E_ARG, "execute_ticks < 0");
    // admission by memory: a query must fit one lane window
    if (msc_query_bytes(q) > o->control->hi) return ctx_fail(o, MSC_E_NOMEM, "query exceeds a lane window");
    q->replan_depth = 0;
    Job job;
    job.q = q;
    job.bind = bind_scene(q->scene);   // the grid of the scene's current tick
    bool refused = false;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        // admission by queue depth: a submission that would wait behind max_pending
        // others is refused (the caller sheds it); replans issued by msc_server_step are not
        refused = S->max_pending && S->queue.size() >= S->max_pending;
        if (!refused) {
            job.ticket = S->next_ticket++;
            *ticket = job.ticket;
            S->submitted[job.ticket] = now_ms();
            S->queue.push_back(std::move(job));
        }
    }
    if (refused) {
        unbind_scene(job.bind);
        return MSC_E_CAPACITY;
    }
    S->cv.notify_one();
    return MSC_OK;
}

msc_status msc_server_poll(msc_ctx* o, uint64_t ticket, int32_t* done) {
    if (!o || !done) return MSC_E_ARG;
    ServerState* S = o->server;
    if (!S) return ctx_fail(o, MSC_E_STATE, "the server is not running");
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->done.find(ticket);
    if (it != S->done.end()) {
        S->done.erase(it);
        *done = 1;
        return MSC_OK;
    }
    if (!S->submitted.count(ticket)) return ctx_fail(o, MSC_E_STATE, "unknown ticket, or its completion was already reported");
    *done = 0;
    return MSC_OK;
}

msc_status msc_server_wait(msc_ctx* o, uint64_t ticket) {
    if (!o) return MSC_E_ARG;
    ServerState* S = o->server;
    if (!S) return ctx_fail(o, MSC_E_STATE, "the server is not running");
    std::unique_lock<std::mutex> lock(S->mu);
    if (!S->done.count(ticket) && !S->submitted.count(ticket))
        return ctx_fail(o, MSC_E_STATE, "unknown ticket, or its completion was already reported");
    S->done_cv.wait(lock, [&] { return S->done.count(ticket) > 0; });
    S->done.erase(ticket);
    return MSC_OK;
}

msc_status msc_server_step(msc_ctx* o, int64_t tick, msc_step_report* report) {
    if (!o) return MSC_E_ARG;
    ServerState* S = o->server;
    if (!S) return ctx_fail(o, MSC_E_STATE, "the server is not running");
    Lane* c = o->control;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    std::vector<Exec> ex;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        if (tick < S->tick) return ctx_fail(o, MSC_E_ARG, "the logical clock does not go backward");
        S->tick = tick;
        ex.swap(S->executing);
    }
    msc_step_report r{};
    // (path, waypoint reached at this tick) of the paths still moving
    std::vector<std::pair<size_t, int>> live;
    for (size_t i = 0; i < ex.size(); ++i) {
        const int64_t w = tick > ex[i].start_tick ? (tick - ex[i].start_tick) / ex[i].tpw : 0;
        if (w >= ex[i].W) {
            ++r.finished;
            continue;
        }
        live.emplace_back(i, (int)w);
    }
    std::vector<std::vector<uint8_t>> valid;
    prof_reset(c, 0u);
    msc_status st = revalidate(c, ex, live, valid);
    if (st != MSC_OK) {
        // keep the paths for the next step
        std::lock_guard<std::mutex> lock(S->mu);
        for (auto& e : ex) S->executing.push_back(std::move(e));
        o->err = c->err;
        return st;
    }
    std::vector<Exec> keep;
    std::vector<Job> jobs;
    std::vector<std::unique_ptr<ReplanRec>> recs;
    for (size_t i = 0; i < live.size(); ++i) {
        Exec& e = ex[live[i].first];
        const int d = live[i].second;
        const std::vector<uint8_t>& v = valid[i];
        r.poses_checked += (int64_t)v.size();
        bool all = true;
        for (uint8_t b : v) all = all && b;
        if (all) {
            keep.push_back(std::move(e));
            continue;
        }
        if (!v[0]) {
            // the arm's current pose is hit: there is no pose to replan from
            ++r.stopped;
            continue;
        }
        // the rest of the path, replanned from the current pose to the same target and
        // kept nearest the rest of the original path; it executes when it is solved
        const int n = e.arm.dof;
        const int W2 = e.W - d;
        auto rec = std::make_unique<ReplanRec>();
        rec->arm = e.arm;
        rec->start.assign(e.rows.begin() + (size_t)d * n, e.rows.begin() + (size_t)(d + 1) * n);
        rec->ref.assign(e.rows.begin() + (size_t)d * n, e.rows.end());
        rec->out.assign((size_t)(W2 + 1) * n, 0);
        msc_query& q = rec->q;
        q.scene = e.scene;
        q.arm = &rec->arm;
        q.kind = 1;
        for (int k = 0; k < 3; ++k) q.target[k] = e.target[k];
        q.start_cdeg = rec->start.data();
        q.waypoints = W2;
        q.max_delta_cdeg = e.max_delta_cdeg;
        q.out = rec->out.data();
        q.status = MSC_E_STATE;
        q.ref_cdeg = rec->ref.data();
        q.execute_ticks = e.tpw;
        q.replan_depth = e.depth + 1;
        rec->issued_ms = now_ms();
        Job job;
        job.q = &rec->q;
        job.rec = rec.get();
        job.bind = bind_scene(e.scene);
        jobs.push_back(std::move(job));
        recs.push_back(std::move(rec));
        ++r.replans;
    }
    {
        std::lock_guard<std::mutex> lock(S->mu);
        for (auto& e : keep) S->executing.push_back(std::move(e));
        // replans go ahead of new requests: the arm is already moving
        for (size_t j = jobs.size(); j-- > 0;) {
            jobs[j].ticket = S->next_ticket++;
            S->replans[jobs[j].ticket] = std::move(recs[j]);
            S->queue.push_front(std::move(jobs[j]));
        }
        r.executing = (int32_t)S->executing.size();
    }
    if (r.replans) S->cv.notify_all();
    if (report) *report = r;
    return MSC_OK;
}

msc_status msc_server_take_replans(msc_ctx* o, msc_query* out, int32_t cap, int32_t* count) {
    if (!o || !count || cap < 0 || (cap && !out)) return MSC_E_ARG;
    ServerState* S = o->server;
    if (!S) return ctx_fail(o, MSC_E_STATE, "the server is not running");
    std::lock_guard<std::mutex> lock(S->mu);
    S->taken.clear();
    int32_t k = 0;
    size_t i = 0;
    for (; i < S->replans_done.size() && k < cap; ++i, ++k) {
        auto it = S->replans.find(S->replans_done[i]);
        out[k] = it->second->q;
        S->taken.push_back(std::move(it->second));
        S->replans.erase(it);
    }
    S->replans_done.erase(S->replans_done.begin(), S->replans_done.begin() + (ptrdiff_t)i);
    *count = k;
    return MSC_OK;
}

msc_status msc_server_stop(msc_ctx* o) {
    if (!o) return MSC_E_ARG;
    ServerState* S = o->server;
    if (!S) return MSC_OK;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto& t : S->threads) t.join();
    delete S;
    o->server = nullptr;
    return MSC_OK;
}

msc_status msc_pose_check(msc_ctx* o, const msc_scene* sc, const msc_arm* arm, const int32_t* poses_cdeg,
                          int64_t count, uint8_t* valid_out, int32_t* end_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;

    MSC_TRY(check_scene(c, sc));
    MSC_TRY(check_arm(c, arm, sc->n));
    if (count < 0 || (count && (!poses_cdeg || !valid_out))) return fail(c, MSC_E_ARG, "bad pose arrays");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    Plan p;
    make_plan(arm, nullptr, p);
    const int64_t chunk = 1 << 20;
    std::vector<int32_t> q;
    for (int64_t b = 0; b < count; b += chunk) {
        begin_call(c);
        int64_t cnt = std::min(chunk, count - b);
        q.assign(poses_cdeg + b * p.n, poses_cdeg + (b + cnt) * p.n);
        for (auto& v : q) {
            if (v % arm->step_cdeg) return fail(c, MSC_E_ARG, "pose angle not a multiple of the step");
            v /= arm->step_cdeg;
        }
        MSC_TRY(pose_check_steps(c, sc, p, q.data(), cnt, valid_out + b, end_out ? end_out + b * 3 : nullptr));
    }
    return MSC_OK;
}

}  // extern "C"

namespace {

// Argument checks of msc_refine / msc_refine_static and the kernel's view of the arm.
msc_status refine_prepare(Lane* c, const msc_arm* arm, const int32_t* poses_cdeg, const double* targets,
                          int64_t count, double* angles_out, int32_t* status_out, RefineArgs& a) {
    MSC_TRY(check_arm(c, arm, 1 << 30));
    const int n = arm->dof;
    if (n < 4 || arm->len_vox[n - 4] != 0 || arm->len_vox[n - 2] != 0 || arm->len_vox[n - 3] <= 0 ||
        arm->len_vox[n - 1] <= 0 || arm->type[n - 4] == arm->type[n - 3] || arm->type[n - 2] == arm->type[n - 1])
        return fail(c, MSC_E_ARG, "the last two segments must each be a zero-length link and a link of the other kind");
    if (count < 0 || (count && (!poses_cdeg || !targets || !angles_out || !status_out)))
        return fail(c, MSC_E_ARG, "bad pose arrays");
    for (int64_t i = 0; i < count * n; ++i)
        if (poses_cdeg[i] % arm->step_cdeg) return fail(c, MSC_E_ARG, "pose angle not a multiple of the step");
    for (int64_t i = 0; i < count * 3; ++i)
        if (!std::isfinite(targets[i])) return fail(c, MSC_E_ARG, "target not finite");
    a = RefineArgs{};
    a.n = n;
    a.q_div = 1;
    for (int k = 0; k < n; ++k) {
        a.type[k] = arm->type[k];
        a.len[k] = (double)arm->len_vox[k];
    }
    for (int d = 0; d < 3; ++d) a.base[d] = (double)arm->base[d];
    a.az0 = arm->az0_cdeg / 100.0;
    a.el0 = arm->el0_cdeg / 100.0;
    a.step = arm->step_cdeg / 100.0;
    return MSC_OK;
}

// Device bytes msc_refine_static needs for `count` poses of n joints: the poses, the
// targets, the angles and the statuses, each region 256-byte aligned.
uint64_t refine_static_bytes(int n, int64_t count) {
    return align_up((uint64_t)count * n * 4) + align_up((uint64_t)count * 24) + align_up((uint64_t)count * n * 8) +
           align_up((uint64_t)count * 4);
}

}  // namespace

extern "C" {

msc_status msc_refine(msc_ctx* o, const msc_arm* arm, const int32_t* poses_cdeg, const double* targets,
                      int64_t count, double* angles_out, int32_t* status_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;

    RefineArgs a;
    MSC_TRY(refine_prepare(c, arm, poses_cdeg, targets, count, angles_out, status_out, a));
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    const int n = a.n;
    // the kernel time of every chunk is kept for msc_get_timings
    prof_reset(c, MSC_PROFILE);
    const int64_t chunk = 1 << 20;
    std::vector<int32_t> q;
    for (int64_t b = 0; b < count; b += chunk) {
        begin_call(c);
        const int64_t cnt = std::min(chunk, count - b);
        q.assign(poses_cdeg + b * n, poses_cdeg + (b + cnt) * n);
        for (auto& v : q) v /= arm->step_cdeg;
        void *d_q, *d_t, *d_a, *d_s;
        MSC_TRY(arena_alloc(c, (uint64_t)cnt * n * 4, &d_q));
        MSC_TRY(arena_alloc(c, (uint64_t)cnt * 24, &d_t));
        MSC_TRY(arena_alloc(c, (uint64_t)cnt * n * 8, &d_a));
        MSC_TRY(arena_alloc(c, (uint64_t)cnt * 4, &d_s));
        HIP_TRY(hipMemcpyAsync(d_q, q.data(), (size_t)cnt * n * 4, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(d_t, targets + b * 3, (size_t)cnt * 24, hipMemcpyHostToDevice, c->stream));
        LAUNCH(MSC_K_REFINE, -1, cnt,
               launch_refine(a, (const int32_t*)d_q, (const double*)d_t, cnt, (double*)d_a, (int32_t*)d_s, c->stream));
        HIP_TRY(hipMemcpyAsync(angles_out + b * n, d_a, (size_t)cnt * n * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(status_out + b, d_s, (size_t)cnt * 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    prof_finish(c);
    return MSC_OK;
}

int64_t msc_refine_static_max(int32_t dof) {
    if (dof < 1 || dof > MSC_MAX_DOF) return 0;
    int64_t lo = 0, hi = (int64_t)(MSC_REFINE_STATIC_BYTES / 64);
    while (lo < hi) {   // largest count whose regions fit the buffer
        const int64_t mid = (lo + hi + 1) / 2;
        if (refine_static_bytes(dof, mid) <= MSC_REFINE_STATIC_BYTES)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

msc_status msc_refine_static(msc_ctx* o, const msc_arm* arm, const int32_t* poses_cdeg, const double* targets,
                             int64_t count, double* angles_out, int32_t* status_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;

    RefineArgs a;
    MSC_TRY(refine_prepare(c, arm, poses_cdeg, targets, count, angles_out, status_out, a));
    const int n = a.n;
    if (count > msc_refine_static_max(n))
        return fail(c, MSC_E_CAPACITY,
                    "msc_refine_static: %lld poses of %d joints exceed its %llu-byte device buffer "
                    "(at most %lld per call)",
                    (long long)count, n, (unsigned long long)MSC_REFINE_STATIC_BYTES,
                    (long long)msc_refine_static_max(n));
    if (count == 0) return MSC_OK;
    char* base = static_scratch(o->device);
    if (!base) return fail(c, MSC_E_STATE, "msc_refine_static: no device buffer address for device %d", o->device);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    // the kernel divides the centidegree values by the step itself: no host copy
    a.q_div = arm->step_cdeg;
    char* d_q = base;
    char* d_t = d_q + align_up((uint64_t)count * n * 4);
    char* d_a = d_t + align_up((uint64_t)count * 24);
    char* d_s = d_a + align_up((uint64_t)count * n * 8);
    HIP_TRY(hipMemcpyAsync(d_q, poses_cdeg, (size_t)count * n * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_t, targets, (size_t)count * 24, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_refine(a, (const int32_t*)d_q, (const double*)d_t, count, (double*)d_a, (int32_t*)d_s,
                          c->stream));
    HIP_TRY(hipMemcpyAsync(angles_out, d_a, (size_t)count * n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(status_out, d_s, (size_t)count * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MSC_OK;
}

msc_status msc_get_stats(msc_ctx* o, msc_stats* out) {
    if (!o || !out) return MSC_E_ARG;
    *out = o->control->stats;
    return MSC_OK;
}

msc_status msc_debug_tables(msc_ctx* o, const msc_arm* arm, int32_t stage, int32_t* off, int32_t* sweep) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;

    MSC_TRY(check_arm(c, arm, 1 << 30));
    if (stage < 0 || stage >= arm->dof || !off || !sweep) return fail(c, MSC_E_ARG, "bad stage or output");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    begin_call(c);
    int na = 36000 / arm->step_cdeg, S = arm->samples;
    TableEntry t;
    MSC_TRY(get_table(c, na, S, arm->len_vox[stage], &t));
    std::vector<short4> ho((size_t)na * na), hs((size_t)na * na * S);
    HIP_TRY(hipMemcpyAsync(ho.data(), t.off, ho.size() * sizeof(short4), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hs.data(), t.sweep, hs.size() * sizeof(short4), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < ho.size(); ++i) {
        off[i * 3] = ho[i].x;
        off[i * 3 + 1] = ho[i].y;
        off[i * 3 + 2] = ho[i].z;
    }
    for (size_t i = 0; i < hs.size(); ++i) {
        sweep[i * 3] = hs[i].x;
        sweep[i * 3 + 1] = hs[i].y;
        sweep[i * 3 + 2] = hs[i].z;
    }
    return MSC_OK;
}

msc_status msc_debug_raster(msc_ctx* o, const msc_scene* sc, uint8_t* occ_out) {
    if (!o) return MSC_E_ARG;
    Lane* c = o->control;

    MSC_TRY(check_scene(c, sc));
    if (!occ_out) return fail(c, MSC_E_ARG, "NULL output");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MSC_E_HIP, "hipSetDevice");
    const int n = sc->n;
    std::vector<uint64_t> w((size_t)n * n * sc->wpr);
    HIP_TRY(hipMemcpyAsync(w.data(), sc->grid, w.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                uint64_t word = w[((size_t)z * n + y) * sc->wpr + (x >> 6)];
                occ_out[((size_t)z * n + y) * n + x] = (uint8_t)((word >> (x & 63)) & 1);
            }
    return MSC_OK;
}

msc_status msc_debug_set(msc_ctx* o, int32_t which, int32_t stage, uint64_t* keys, uint64_t cap, uint64_t* count) {
    if (!o || !count) return MSC_E_ARG;
    Lane* c = o->control;

    if (which == 2) {
        for (auto& kv : c->captured)
            if (kv.first.first == 2) {
                stage = kv.first.second;
                break;
            }
    }
    auto it = c->captured.find({which, stage});
    if (it == c->captured.end()) return fail(c, MSC_E_STATE, "set %d/%d was not captured", which, stage);
    *count = it->second.size();
    if (keys) std::memcpy(keys, it->second.data(), std::min<uint64_t>(cap, it->second.size()) * 8);
    return MSC_OK;
}

const char* msc_last_error(msc_ctx* o) {
    if (!o) return "NULL context";
    if (!o->err.empty()) return o->err.c_str();
    return o->control->err.c_str();
}

}  // extern "C"
