// Host runtime and C ABI of libmsc: argument checks, the device workspace arena, the
// stage schedule of the reach search and the path search.  All arithmetic of the
// method runs in the kernels of msc_kernels.hip; this file plans memory, launches
// and copies results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "msc.h"
#include "msc_common.h"

using namespace msc;

namespace {

constexpr uint64_t kAlign = 256;
constexpr size_t kStagingBytes = 1 << 20;
constexpr int kCounters = 512;

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
};

}  // namespace

struct msc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    uint64_t lo = 0;   // per-call region grows up from 0
    uint64_t hi = 0;   // persistent region grows down from ws_bytes
    std::string err;
    std::map<std::tuple<int, int, int>, TableEntry> tables;
    unsigned long long* counters = nullptr;  // device, persistent
    int next_counter = 0;
    unsigned long long* ovf = nullptr;       // overflow counter of the current call
    char* staging = nullptr;                 // pinned host
    size_t staging_used = 0;
    msc_stats stats{};
    std::map<std::pair<int, int>, std::vector<uint64_t>> captured;
    int captured_n = 0;
};

struct msc_scene {
    msc_ctx* ctx = nullptr;
    int n = 0, wpr = 0, dilate = 0;
    uint64_t* grid = nullptr;
    uint64_t bytes = 0;
};

namespace {

msc_status fail(msc_ctx* c, msc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

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

msc_status arena_alloc(msc_ctx* c, uint64_t bytes, void** out) {
    uint64_t b = align_up(bytes ? bytes : 1);
    if (c->lo + b > c->hi) {
        return fail(c, MSC_E_NOMEM, "workspace exhausted: need %llu more bytes (used %llu of %llu)",
                    (unsigned long long)b, (unsigned long long)c->lo, (unsigned long long)c->hi);
    }
    *out = c->ws + c->lo;
    c->lo += b;
    return MSC_OK;
}

msc_status persist_alloc(msc_ctx* c, uint64_t bytes, void** out) {
    uint64_t b = align_up(bytes ? bytes : 1);
    if (c->hi < b || c->hi - b < c->lo) return fail(c, MSC_E_NOMEM, "workspace exhausted (persistent tables)");
    c->hi -= b;
    *out = c->ws + c->hi;
    return MSC_OK;
}

void begin_call(msc_ctx* c) {
    c->lo = 0;
    c->staging_used = 0;
    c->next_counter = 0;
    c->err.clear();
}

// Upload a small host array through the pinned staging buffer (no host sync).
msc_status upload(msc_ctx* c, const void* src, size_t bytes, void** dev) {
    size_t b = (bytes + 255) & ~(size_t)255;
    if (c->staging_used + b > kStagingBytes - 4096) return fail(c, MSC_E_NOMEM, "staging buffer exhausted");
    char* h = c->staging + c->staging_used;
    c->staging_used += b;
    std::memcpy(h, src, bytes);
    MSC_TRY(arena_alloc(c, bytes, dev));
    HIP_TRY(hipMemcpyAsync(*dev, h, bytes, hipMemcpyHostToDevice, c->stream));
    return MSC_OK;
}

unsigned long long* take_counter(msc_ctx* c) {
    if (c->next_counter >= kCounters) return nullptr;
    return c->counters + c->next_counter++;
}

msc_status read_counter(msc_ctx* c, unsigned long long* dev, uint64_t* out) {
    unsigned long long* h = (unsigned long long*)(c->staging + kStagingBytes - 64);
    HIP_TRY(hipMemcpyAsync(h, dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *out = *h;
    return MSC_OK;
}

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
    int split;   // -1 adaptive
};

msc_status check_arm(msc_ctx* c, const msc_arm* arm, int grid_n) {
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
    p.split = -1;
}

msc_status get_table(msc_ctx* c, int na, int S, int L, TableEntry* out) {
    auto key = std::make_tuple(na, S, L);
    auto it = c->tables.find(key);
    if (it != c->tables.end()) {
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
    c->tables[key] = t;
    *out = t;
    return MSC_OK;
}

GridView grid_view(const msc_scene* s) { return GridView{s->grid, s->n, s->wpr}; }

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
msc_status make_set(msc_ctx* c, const Plan& p, const Box& box, uint64_t upper, int fast_ia, bool force_dense,
                    StageSet& s) {
    const uint64_t na2 = (uint64_t)p.na * p.na;
    uint64_t dense_words = box.empty() ? 0 : (box.voxels() * na2 + 63) / 64 + 1;
    uint64_t hash_slots = pow2_at_least(std::max<uint64_t>(2 * upper, 64));
    bool dense = !box.empty() && (force_dense || dense_words <= hash_slots);
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
        MSC_TRY(arena_alloc(c, dense_words * 8, &mem));
        s.view.words = (uint64_t*)mem;
        HIP_TRY(launch_fill(s.view.words, dense_words, 0ull, c->stream));
    } else {
        s.view.kind = kHash;
        s.view.cap = hash_slots;
        MSC_TRY(arena_alloc(c, hash_slots * 8, &mem));
        s.view.words = (uint64_t*)mem;
        HIP_TRY(launch_fill(s.view.words, hash_slots, kEmpty, c->stream));
    }
    return MSC_OK;
}

msc_status ensure_list(msc_ctx* c, StageSet& s) {
    if (s.listed) return MSC_OK;
    void* mem;
    MSC_TRY(arena_alloc(c, std::max<uint64_t>(s.count, 1) * 8, &mem));
    s.list = (uint64_t*)mem;
    unsigned long long* ctr = take_counter(c);
    if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
    HIP_TRY(launch_compact(s.view, s.list, s.count, ctr, c->ovf, c->stream));
    s.listed = true;
    return MSC_OK;
}

// Copy a set's members to the host as sorted keys ((z*N + y)*N + x) << 16 | ia << 8 | ie.
msc_status capture_set(msc_ctx* c, StageSet& s, int N, int which, int stage) {
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

msc_status check_overflow(msc_ctx* c, unsigned long long* ovf, const char* what) {
    uint64_t v = 0;
    MSC_TRY(read_counter(c, ovf, &v));
    if (v) return fail(c, MSC_E_CAPACITY, "%s overflowed (%llu states without room)", what, (unsigned long long)v);
    return MSC_OK;
}

// The staged reach search.  Returns MSC_OK with up to `want` solutions (steps) in the
// canonical order, or MSC_NO_REACH.
msc_status run_reach(msc_ctx* c, const msc_scene* sc, const Plan& p, int want, bool capture, ReachOut& out) {
    const int n = p.n, na = p.na, N = sc->n;
    const GridView g = grid_view(sc);
    std::memset(&c->stats, 0, sizeof c->stats);
    c->stats.dof = n;
    c->captured.clear();
    c->captured_n = N;
    out = ReachOut();

    HIP_TRY(launch_fill((uint64_t*)c->counters, kCounters, 0ull, c->stream));
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
        void *d_type, *d_lo, *d_hi, *scratch, *m1, *m2;
        MSC_TRY(upload(c, p.type, sizeof(int32_t) * n, &d_type));
        MSC_TRY(upload(c, p.lo, sizeof(int32_t) * n, &d_lo));
        MSC_TRY(upload(c, p.hi, sizeof(int32_t) * n, &d_hi));
        MSC_TRY(arena_alloc(c, (uint64_t)(n + 1) * na * na, &scratch));
        MSC_TRY(arena_alloc(c, (uint64_t)(n + 1) * na * 4 * 8, &m1));
        MSC_TRY(arena_alloc(c, (uint64_t)(n + 1) * na * 4 * 8, &m2));
        rows_ie = (uint64_t*)m1;
        rows_ia = (uint64_t*)m2;
        HIP_TRY(launch_orient(n, na, p.ia0, p.ie0, (const int32_t*)d_type, (const int32_t*)d_lo,
                              (const int32_t*)d_hi, (uint8_t*)scratch, rows_ie, rows_ia, c->stream));
    }
    auto rows_for = [&](int stage, int yaw) -> const uint64_t* {
        if (!p.prune) return nullptr;
        return (yaw ? rows_ia : rows_ie) + (size_t)stage * na * 4;
    };

    std::vector<StageSet> F(n + 1), B(n + 1);
    std::vector<Box> box(n + 1);
    for (int k = 0; k <= n; ++k) box[k] = stage_box(p, N, R, k);

    // Seeds.
    {
        Box b0{p.base[0], p.base[1], p.base[2], 1, 1, 1};
        MSC_TRY(make_set(c, p, b0, 1, 0, false, F[0]));
        unsigned long long* ctr = take_counter(c);
        HIP_TRY(launch_seed_fwd(F[0].view, g, p.base[0], p.base[1], p.base[2], p.ia0, p.ie0, ctr, c->stream));
        MSC_TRY(read_counter(c, ctr, &F[0].count));
        Box bn{p.target[0], p.target[1], p.target[2], 1, 1, 1};
        int fast = p.type[n - 1] == MSC_YAW ? 1 : 0;
        MSC_TRY(make_set(c, p, bn, (uint64_t)na * na, fast, true, B[n]));
        ctr = take_counter(c);
        HIP_TRY(launch_seed_bwd(B[n].view, g, p.target[0], p.target[1], p.target[2], rows_for(n, 0), p.prune, ctr,
                                c->stream));
        MSC_TRY(read_counter(c, ctr, &B[n].count));
    }
    bool empty = F[0].count == 0 || B[n].count == 0;
    int kf = 0, kb = n;
    unsigned long long* ovf = c->ovf;
    while (!empty && kf < kb) {
        bool forward;
        if (p.split >= 0) {
            forward = kf < p.split;
        } else {
            double cf = (double)F[kf].count * (p.hi[kf] - p.lo[kf] + 1);
            double cb = (double)B[kb].count * 3.0;
            forward = cf <= cb;
        }
        if (forward) {
            const int k = kf + 1;  // joint k-1 (0-based) lays segment k
            MSC_TRY(ensure_list(c, F[kf]));
            uint64_t upper = F[kf].count * (uint64_t)(p.hi[k - 1] - p.lo[k - 1] + 1);
            MSC_TRY(make_set(c, p, box[k], upper, 0, false, F[k]));
            int64_t rt = 0;
            for (int j = k; j < n; ++j) rt += R[j];
            long long r2 = p.prune ? (long long)(rt * rt) : -1;
            unsigned long long* ctr = take_counter(c);
            if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
            HIP_TRY(launch_expand_fwd(F[kf].list, F[kf].count, F[k].view, g, jv[k - 1], p.target[0], p.target[1],
                                      p.target[2], r2, ctr, ovf, c->stream));
            MSC_TRY(read_counter(c, ctr, &F[k].count));
            kf = k;
            empty = F[k].count == 0;
        } else {
            const int k = kb;  // joint k-1 (0-based) lays segment k; produce B_{k-1}
            MSC_TRY(ensure_list(c, B[kb]));
            uint64_t upper = B[kb].count * (uint64_t)(p.hi[k - 1] - p.lo[k - 1] + 1);
            int yaw = p.type[k - 1] == MSC_YAW ? 1 : 0;
            MSC_TRY(make_set(c, p, box[k - 1], upper, yaw, false, B[k - 1]));
            int64_t rb = 0;
            for (int j = 0; j < k - 1; ++j) rb += R[j];
            long long r2 = p.prune ? (long long)(rb * rb) : -1;
            unsigned long long* ctr = take_counter(c);
            if (!ctr) return fail(c, MSC_E_CAPACITY, "out of counters");
            HIP_TRY(launch_expand_bwd(B[kb].list, B[kb].count, B[k - 1].view, g, jv[k - 1], p.base[0], p.base[1],
                                      p.base[2], r2, rows_for(k - 1, yaw), ctr, ovf, c->stream));
            MSC_TRY(read_counter(c, ctr, &B[k - 1].count));
            kb = k - 1;
            empty = B[k - 1].count == 0;
        }
    }
    MSC_TRY(check_overflow(c, ovf, "a stage set"));
    const int m = kf;
    c->stats.split_m = m;
    for (int k = 0; k <= n; ++k) {
        c->stats.fwd_count[k] = F[k].used ? (int64_t)F[k].count : -1;
        c->stats.bwd_count[k] = B[k].used ? (int64_t)B[k].count : -1;
        c->stats.fwd_dense[k] = F[k].used && F[k].view.kind == kDense;
        c->stats.bwd_dense[k] = B[k].used && B[k].view.kind == kDense;
    }
    if (capture) {
        for (int k = 0; k <= n; ++k) {
            if (F[k].used) MSC_TRY(capture_set(c, F[k], N, 0, k));
            if (B[k].used) MSC_TRY(capture_set(c, B[k], N, 1, k));
        }
    }
    if (empty) return MSC_NO_REACH;

    // Join and D marking.
    MSC_TRY(ensure_list(c, F[m]));
    unsigned long long* jc = take_counter(c);
    HIP_TRY(launch_join(F[m].list, F[m].count, F[m].view, B[m].view, jc, c->stream));
    uint64_t joined = 0;
    MSC_TRY(read_counter(c, jc, &joined));
    c->stats.join_count = (int64_t)joined;
    if (capture) {
        StageSet tmp = F[m];
        tmp.count = F[m].count;
        MSC_TRY(capture_set(c, tmp, N, 2, m));
        c->captured[{3, m}] = c->captured[{2, m}];
    }
    if (joined == 0) return MSC_NO_REACH;
    for (int k = m; k >= 1; --k) {
        MSC_TRY(ensure_list(c, F[k - 1]));
        unsigned long long* dc = take_counter(c);
        HIP_TRY(launch_dmark(F[k - 1].list, F[k - 1].count, F[k - 1].view, F[k].view, g, jv[k - 1], dc, c->stream));
        if (capture) MSC_TRY(capture_set(c, F[k - 1], N, 3, k - 1));
    }

    // Canonical reach poses.
    std::vector<SetView> sets(n + 1);
    for (int k = 0; k <= n; ++k) sets[k] = (k <= m) ? F[k].view : B[k].view;
    void *d_sets, *d_joints, *d_sols, *d_nsol;
    MSC_TRY(upload(c, sets.data(), sizeof(SetView) * (n + 1), &d_sets));
    MSC_TRY(upload(c, jv.data(), sizeof(JointView) * n, &d_joints));
    MSC_TRY(arena_alloc(c, (uint64_t)want * n * 4, &d_sols));
    MSC_TRY(arena_alloc(c, 4, &d_nsol));
    DfsArgs da{};
    da.sets = (const SetView*)d_sets;
    da.joints = (const JointView*)d_joints;
    da.g = g;
    da.n = n;
    da.m = m;
    da.na = na;
    da.want = want;
    for (int k = 0; k < n; ++k) da.ref[k] = p.ref[k];
    da.root = pack_key(p.base[0], p.base[1], p.base[2], p.ia0, p.ie0);
    da.sols = (int32_t*)d_sols;
    da.nsol = (int32_t*)d_nsol;
    HIP_TRY(launch_dfs(da, c->stream));
    int32_t nsol = 0;
    HIP_TRY(hipMemcpyAsync(&nsol, d_nsol, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    MSC_TRY(check_overflow(c, ovf, "a stage set"));
    if (nsol <= 0) return fail(c, MSC_E_STATE, "join not empty but no pose traced");
    out.nsol = std::min(nsol, want);
    out.sols.resize((size_t)out.nsol * n);
    HIP_TRY(hipMemcpyAsync(out.sols.data(), d_sols, out.sols.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MSC_OK;
}

msc_status joint_views(msc_ctx* c, const Plan& p, std::vector<JointView>& jv) {
    jv.resize(p.n);
    for (int k = 0; k < p.n; ++k) {
        TableEntry t;
        MSC_TRY(get_table(c, p.na, p.S, p.len[k], &t));
        jv[k] = JointView{t.off, t.sweep, p.type[k], p.lo[k], p.hi[k], p.S};
    }
    return MSC_OK;
}

msc_status pose_check_steps(msc_ctx* c, const msc_scene* sc, const Plan& p, const int32_t* q_steps, int64_t count,
                            uint8_t* valid, int32_t* ends) {
    std::vector<JointView> jv;
    MSC_TRY(joint_views(c, p, jv));
    void *d_joints, *d_q, *d_valid, *d_ends = nullptr;
    MSC_TRY(upload(c, jv.data(), sizeof(JointView) * p.n, &d_joints));
    MSC_TRY(arena_alloc(c, (uint64_t)count * p.n * 4, &d_q));
    MSC_TRY(arena_alloc(c, (uint64_t)count, &d_valid));
    if (ends) MSC_TRY(arena_alloc(c, (uint64_t)count * 12, &d_ends));
    HIP_TRY(hipMemcpyAsync(d_q, q_steps, (size_t)count * p.n * 4, hipMemcpyHostToDevice, c->stream));
    PoseArgs a{};
    a.joints = (const JointView*)d_joints;
    a.g = grid_view(sc);
    a.n = p.n;
    a.na = p.na;
    a.bx = p.base[0];
    a.by = p.base[1];
    a.bz = p.base[2];
    a.ia0 = p.ia0;
    a.ie0 = p.ie0;
    HIP_TRY(launch_pose_check(a, (const int32_t*)d_q, count, (uint8_t*)d_valid, (int32_t*)d_ends, c->stream));
    HIP_TRY(hipMemcpyAsync(valid, d_valid, (size_t)count, hipMemcpyDeviceToHost, c->stream));
    if (ends) HIP_TRY(hipMemcpyAsync(ends, d_ends, (size_t)count * 12, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MSC_OK;
}

msc_status check_scene(msc_ctx* c, const msc_scene* s) {
    if (!s) return fail(c, MSC_E_ARG, "scene is NULL");
    if (s->ctx != c) return fail(c, MSC_E_ARG, "scene belongs to another context");
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
extern "C" {

void msc_opts_default(msc_opts* o) {
    if (!o) return;
    o->split_m = -1;
    o->tube_r0 = 1;
    o->tube_r1 = 2;
    o->reach_retries = 4;
    o->flags = 0;
}

msc_status msc_ctx_create(int device, void* hip_stream, void* dev_workspace, uint64_t ws_bytes, msc_ctx** out) {
    if (!out || !dev_workspace) return MSC_E_ARG;
    if (ws_bytes < (64ull << 20)) return MSC_E_ARG;
    if ((uintptr_t)dev_workspace % kAlign) return MSC_E_ARG;
    msc_ctx* c = new (std::nothrow) msc_ctx();
    if (!c) return MSC_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)dev_workspace;
    c->ws_bytes = ws_bytes;
    c->hi = ws_bytes;
    if (hipSetDevice(device) != hipSuccess || hipHostMalloc((void**)&c->staging, kStagingBytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return MSC_E_HIP;
    }
    void* p;
    if (persist_alloc(c, kCounters * sizeof(unsigned long long), &p) != MSC_OK) {
        (void)hipHostFree(c->staging);
        delete c;
        return MSC_E_NOMEM;
    }
    c->counters = (unsigned long long*)p;
    *out = c;
    return MSC_OK;
}

msc_status msc_ctx_destroy(msc_ctx* c) {
    if (!c) return MSC_E_ARG;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->staging) (void)hipHostFree(c->staging);
    delete c;
    return MSC_OK;
}

uint64_t msc_scene_bytes(int32_t n) {
    if (n <= 0) return 0;
    uint64_t wpr = ((uint64_t)n + 63) / 64;
    return (uint64_t)n * n * wpr * 8;
}

msc_status msc_scene_create(msc_ctx* c, int32_t n, int32_t dilate_r, const msc_box* boxes, int32_t nbox,
                            const msc_sphere* spheres, int32_t nsph, void* dev_grid, uint64_t grid_bytes,
                            msc_scene** out) {
    if (!c) return MSC_E_ARG;
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
    void *db, *ds;
    MSC_TRY(upload(c, hb.data(), hb.size() * 4, &db));
    MSC_TRY(upload(c, hs.data(), hs.size() * 4, &ds));
    msc_scene* s = new (std::nothrow) msc_scene();
    if (!s) return fail(c, MSC_E_NOMEM, "host allocation");
    s->ctx = c;
    s->n = n;
    s->wpr = (n + 63) / 64;
    s->dilate = dilate_r;
    s->grid = (uint64_t*)dev_grid;
    s->bytes = grid_bytes;
    hipError_t e = launch_raster(s->grid, n, s->wpr, dilate_r, (const int32_t*)db, nbox, (const int32_t*)ds, nsph,
                                 c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete s;
        return fail(c, MSC_E_HIP, "raster: %s", hipGetErrorString(e));
    }
    *out = s;
    return MSC_OK;
}

msc_status msc_scene_destroy(msc_scene* s) {
    if (!s) return MSC_E_ARG;
    delete s;
    return MSC_OK;
}

msc_status msc_reach(msc_ctx* c, const msc_scene* sc, const msc_arm* arm, const int32_t target[3],
                     const msc_opts* opts, int32_t* angles_out) {
    if (!c) return MSC_E_ARG;
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
    p.split = o.split_m;
    ReachOut r;
    msc_status st = run_reach(c, sc, p, 1, (o.flags & MSC_CAPTURE_SETS) != 0, r);
    if (st != MSC_OK) return st;
    for (int k = 0; k < p.n; ++k) angles_out[k] = r.sols[k] * arm->step_cdeg;
    return MSC_OK;
}

msc_status msc_path(msc_ctx* c, const msc_scene* sc, const msc_arm* arm, const int32_t* start_cdeg,
                    const int32_t target[3], int32_t waypoints, int32_t max_delta_cdeg, const msc_opts* opts,
                    int32_t* path_out) {
    if (!c) return MSC_E_ARG;
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
    p.split = o.split_m;
    const int n = p.n;
    const int delta = max_delta_cdeg / arm->step_cdeg;
    int start[kMaxDof];
    for (int k = 0; k < n; ++k) {
        if (start_cdeg[k] % arm->step_cdeg) return fail(c, MSC_E_ARG, "start angle %d not a multiple of the step", k);
        start[k] = start_cdeg[k] / arm->step_cdeg;
        if (start[k] < p.lo[k] || start[k] > p.hi[k]) return fail(c, MSC_E_ARG, "start angle %d outside its limits", k);
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
    void* d_joints;
    MSC_TRY(upload(c, jv.data(), sizeof(JointView) * n, &d_joints));
    const uint64_t mark = c->lo;
    int radii[2] = {o.tube_r0, o.tube_r1};
    int nr = o.tube_r1 == o.tube_r0 ? 1 : 2;
    std::vector<int32_t> path((size_t)(waypoints + 1) * n);
    for (int i = 0; i < r.nsol; ++i) {
        for (int ri = 0; ri < nr; ++ri) {
            c->lo = mark;
            const int rad = radii[ri];
            uint64_t slab = 1;
            for (int k = 0; k < n; ++k) {
                slab *= (uint64_t)(2 * rad + 1);
                if (slab > (1ull << 28)) return fail(c, MSC_E_CAPACITY, "tube of radius %d too large", rad);
            }
            TubeArgs ta{};
            ta.joints = (const JointView*)d_joints;
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
                ta.goal[k] = r.sols[(size_t)i * n + k];
                ta.lim_lo[k] = lim_lo[k];
                ta.lim_hi[k] = lim_hi[k];
            }
            ta.slab = slab;
            void *d_valid, *d_reach, *d_t0, *d_t1, *d_path, *d_status;
            uint64_t cells = (uint64_t)(waypoints + 1) * slab;
            MSC_TRY(arena_alloc(c, cells, &d_valid));
            MSC_TRY(arena_alloc(c, cells, &d_reach));
            MSC_TRY(arena_alloc(c, slab, &d_t0));
            MSC_TRY(arena_alloc(c, slab, &d_t1));
            MSC_TRY(arena_alloc(c, path.size() * 4, &d_path));
            MSC_TRY(arena_alloc(c, 4, &d_status));
            HIP_TRY(launch_tube_valid(ta, (uint8_t*)d_valid, c->stream));
            HIP_TRY(launch_tube_solve(ta, (const uint8_t*)d_valid, (uint8_t*)d_reach, (uint8_t*)d_t0, (uint8_t*)d_t1,
                                      (int32_t*)d_path, (int32_t*)d_status, c->stream));
            int32_t ok2 = 0;
            HIP_TRY(hipMemcpyAsync(&ok2, d_status, 4, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            c->stats.attempts++;
            if (ok2) {
                HIP_TRY(hipMemcpyAsync(path.data(), d_path, path.size() * 4, hipMemcpyDeviceToHost, c->stream));
                HIP_TRY(hipStreamSynchronize(c->stream));
                for (size_t j = 0; j < path.size(); ++j) path_out[j] = path[j] * arm->step_cdeg;
                c->stats.tube_r = rad;
                c->stats.reach_index = i;
                return MSC_OK;
            }
        }
    }
    return MSC_NO_PATH;
}

msc_status msc_pose_check(msc_ctx* c, const msc_scene* sc, const msc_arm* arm, const int32_t* poses_cdeg,
                          int64_t count, uint8_t* valid_out, int32_t* end_out) {
    if (!c) return MSC_E_ARG;
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

msc_status msc_get_stats(msc_ctx* c, msc_stats* out) {
    if (!c || !out) return MSC_E_ARG;
    *out = c->stats;
    return MSC_OK;
}

msc_status msc_debug_tables(msc_ctx* c, const msc_arm* arm, int32_t stage, int32_t* off, int32_t* sweep) {
    if (!c) return MSC_E_ARG;
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

msc_status msc_debug_raster(msc_ctx* c, const msc_scene* sc, uint8_t* occ_out) {
    if (!c) return MSC_E_ARG;
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

msc_status msc_debug_set(msc_ctx* c, int32_t which, int32_t stage, uint64_t* keys, uint64_t cap, uint64_t* count) {
    if (!c || !count) return MSC_E_ARG;
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

const char* msc_last_error(msc_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

}  // extern "C"
