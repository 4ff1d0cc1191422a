// HIP kernels of the staged reach / path solver (gfx950, wave64).
//
// The search works on states (joint voxel, orientation) after each segment.  A
// segment is laid along the global direction of its orientation, its S sample
// points are rounded to voxels and tested against the bit-packed occupancy grid
// (paper, "Testing for collisions"); forward stages expand from the root, backward
// stages from the target, and the two sets are intersected ("The gap in gMS",
// "The procedure for IK solution").  Everything here is integer / bitwise work: no
// kernel is a dense contraction, so none uses the matrix cores.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

#include "msc_common.h"

namespace msc {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrap_na(int v, int na) {
    // joint angles stay within one turn, so v is almost always in (-na, 2 na)
    v += v < 0 ? na : 0;
    v -= v >= na ? na : 0;
    if ((unsigned)v >= (unsigned)na) {
        v %= na;
        v += v < 0 ? na : 0;
    }
    return v;
}


__device__ __forceinline__ bool cell_free(const GridView& g, int x, int y, int z) {
    if ((unsigned)x >= (unsigned)g.n || (unsigned)y >= (unsigned)g.n || (unsigned)z >= (unsigned)g.n)
        return false;
    uint64_t w = g.occ[((size_t)z * g.n + y) * g.wpr + (x >> 6)];
    return ((w >> (x & 63)) & 1ull) == 0;
}

// Segment of joint j laid from (x, y, z) along orientation o: clear when every
// sample point is a free voxel inside the grid.
__device__ __forceinline__ bool segment_clear(const GridView& g, const JointView& j, int o, int x, int y,
                                              int z) {
    const short4* sw = j.sweep + (size_t)o * j.S;
    for (int s = j.S - 1; s >= 0; --s) {
        short4 d = sw[s];
        if (!cell_free(g, x + d.x, y + d.y, z + d.z)) return false;
    }
    return true;
}

// Same test with every load issued before any is checked (two memory round trips:
// the sample offsets, then the occupancy words).  The loads are unconditional (an
// out-of-grid sample reads word 0 and is then rejected), so that they can all be in
// flight together.
__device__ __forceinline__ bool segment_clear_all(const GridView& g, const JointView& j, int o, int x, int y,
                                                  int z) {
    if (j.S == 8) {
        // 8 short4 sample offsets = 4 x 16 bytes (the table rows are 64-byte aligned)
        const uint4* sw4 = reinterpret_cast<const uint4*>(j.sweep + (size_t)o * 8);
        uint4 q[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) q[t] = sw4[t];
        uint64_t w[8];
        int bit[8];
        bool in[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t xy = (t & 1) ? q[t >> 1].z : q[t >> 1].x;
            const uint32_t zw = (t & 1) ? q[t >> 1].w : q[t >> 1].y;
            const int px = x + (int)(int16_t)(xy & 0xffffu);
            const int py = y + (int)(int16_t)(xy >> 16);
            const int pz = z + (int)(int16_t)(zw & 0xffffu);
            in[t] = (unsigned)px < (unsigned)g.n && (unsigned)py < (unsigned)g.n && (unsigned)pz < (unsigned)g.n;
            const size_t idx = in[t] ? ((size_t)pz * g.n + py) * g.wpr + (px >> 6) : 0;
            w[t] = g.occ[idx];
            bit[t] = px & 63;
        }
        bool clear = true;
#pragma unroll
        for (int t = 0; t < 8; ++t) clear = clear && in[t] && !((w[t] >> bit[t]) & 1ull);
        return clear;
    }
    const short4* sw = j.sweep + (size_t)o * j.S;
    for (int s0 = 0; s0 < j.S; s0 += 8) {
        short4 d[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) d[t] = sw[s0 + t < j.S ? s0 + t : 0];
        uint64_t w[8];
        int bit[8];
        bool in[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int px = x + d[t].x, py = y + d[t].y, pz = z + d[t].z;
            in[t] = (unsigned)px < (unsigned)g.n && (unsigned)py < (unsigned)g.n && (unsigned)pz < (unsigned)g.n;
            const size_t idx = in[t] ? ((size_t)pz * g.n + py) * g.wpr + (px >> 6) : 0;
            w[t] = g.occ[idx];
            bit[t] = px & 63;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (s0 + t >= j.S) break;
            if (!in[t] || ((w[t] >> bit[t]) & 1ull)) return false;
        }
    }
    return true;
}

__device__ __forceinline__ bool dense_bit(const SetView& s, int x, int y, int z, int ia, int ie,
                                          uint64_t& bit) {
    int dx = x - s.x0, dy = y - s.y0, dz = z - s.z0;
    if ((unsigned)dx >= (unsigned)s.nx || (unsigned)dy >= (unsigned)s.ny || (unsigned)dz >= (unsigned)s.nz)
        return false;
    uint64_t vox = ((uint64_t)dz * s.ny + dy) * s.nx + dx;
    int o = s.fast_ia ? ie * s.na + ia : ia * s.na + ie;
    bit = vox * (uint64_t)(s.na * s.na) + (uint64_t)o;
    return true;
}

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 1 = inserted, 0 = already present, -1 = table full.
__device__ __forceinline__ int hash_insert(const SetView& s, uint64_t key) {
    const uint64_t mask = s.cap - 1;
    uint64_t h = mix64(key) & mask;
    for (uint64_t p = 0; p < s.cap; ++p) {
        uint64_t cur = load_relaxed(&s.words[h]);
        if (cur == kEmpty) {
            uint64_t prev = atomicCAS((unsigned long long*)&s.words[h], (unsigned long long)kEmpty,
                                      (unsigned long long)key);
            if (prev == kEmpty) return 1;
            cur = prev;
        }
        if ((cur & ~kDead) == key) return 0;
        h = (h + 1) & mask;
    }
    return -1;
}

__device__ __forceinline__ int64_t hash_find(const SetView& s, uint64_t key) {
    const uint64_t mask = s.cap - 1;
    uint64_t h = mix64(key) & mask;
    for (uint64_t p = 0; p < s.cap; ++p) {
        uint64_t cur = load_relaxed(&s.words[h]);
        if (cur == kEmpty) return -1;
        if ((cur & ~kDead) == key) return (int64_t)h;
        h = (h + 1) & mask;
    }
    return -1;
}

// 1 = inserted, 0 = already present, -1 = no room (outside the dense box / table full).
__device__ __forceinline__ int set_insert(const SetView& s, int x, int y, int z, int ia, int ie) {
    if (s.kind == kDense) {
        uint64_t bit;
        if (!dense_bit(s, x, y, z, ia, ie, bit)) return -1;
        uint64_t m = 1ull << (bit & 63);
        uint64_t old = atomicOr((unsigned long long*)&s.words[bit >> 6], (unsigned long long)m);
        return (old & m) ? 0 : 1;
    }
    return hash_insert(s, pack_key(x, y, z, ia, ie));
}

__device__ __forceinline__ bool set_member(const SetView& s, uint64_t key) {
    if (s.kind == kDense) {
        int x, y, z, ia, ie;
        unpack_key(key, x, y, z, ia, ie);
        uint64_t bit;
        if (!dense_bit(s, x, y, z, ia, ie, bit)) return false;
        return (load_relaxed(&s.words[bit >> 6]) >> (bit & 63)) & 1ull;
    }
    const uint64_t mask = s.cap - 1;
    uint64_t h = mix64(key) & mask;
    for (uint64_t p = 0; p < s.cap; ++p) {
        uint64_t cur = load_relaxed(&s.words[h]);
        if (cur == kEmpty) return false;
        if ((cur & ~kDead) == key) return (cur & kDead) == 0;
        h = (h + 1) & mask;
    }
    return false;
}

__device__ __forceinline__ void set_remove(const SetView& s, uint64_t key) {
    if (s.kind == kDense) {
        int x, y, z, ia, ie;
        unpack_key(key, x, y, z, ia, ie);
        uint64_t bit;
        if (!dense_bit(s, x, y, z, ia, ie, bit)) return;
        atomicAnd((unsigned long long*)&s.words[bit >> 6], ~(unsigned long long)(1ull << (bit & 63)));
        return;
    }
    int64_t slot = hash_find(s, key);
    if (slot >= 0) atomicOr((unsigned long long*)&s.words[slot], (unsigned long long)kDead);
}

// Block-wide sum of a per-thread count, one atomic per block.
__device__ void block_add(unsigned long long v, unsigned long long* dst) {
    __shared__ unsigned long long part[kBlock / 64];
    __syncthreads();  // the array may still be read by a previous call
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        if (t && dst) atomicAdd(dst, t);
    }
}

// Bits lo..hi (inclusive, 0 <= lo <= hi < 256) of a 256-bit mask.
__device__ __forceinline__ void mask_range(uint64_t m[4], int lo, int hi) {
    for (int w = 0; w < 4; ++w) {
        int a = lo - 64 * w, b = hi - 64 * w;
        if (b < 0 || a > 63) continue;
        a = a < 0 ? 0 : a;
        b = b > 63 ? 63 : b;
        uint64_t top = (b == 63) ? ~0ull : ((1ull << (b + 1)) - 1);
        uint64_t bot = (1ull << a) - 1;
        m[w] |= top & ~bot;
    }
}

// Lanes that share one state when a kernel tries a joint's whole window for it (a
// power of two G <= 64; lane l of a group takes the angles lo + l, lo + l + G, ...).
// Small inputs get a lane per angle, so that the launch still fills the device; large
// ones fewer lanes per state, so that lanes are not left idle by a window that is not
// a power of two.
int group_log2_for(uint64_t count, int nA) {
    int cap = 0;
    while ((1 << cap) < nA && cap < 6) ++cap;
    int lg = 0;
    while (lg < cap && count * (1ull << lg) < (1ull << 20)) ++lg;
    return lg;
}

// Events for the next set-expansion launch (host thread local): when set, the launch
// carries them on its own dispatch (hipExtLaunchKernelGGL), so they time the kernel
// itself rather than the kernel plus the gap before it.
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
thread_local bool t_ev_used = false;

template <typename K, typename... A>
void launch_timed(K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t st, A... args) {
    if (t_ev_start) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, t_ev_start, t_ev_stop, 0u, args...);
        t_ev_used = true;
        t_ev_start = t_ev_stop = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
    }
}

uint32_t grid_for(uint64_t work, uint32_t block = kBlock, uint32_t max_blocks = 16384) {
    uint64_t b = (work + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (uint32_t)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fill (used instead of a memset so that every clear is a kernel).
// ---------------------------------------------------------------------------
__global__ void k_fill(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// 16-byte aligned buffers: pairs of words per store; the odd last word by one thread.
__global__ void k_fill16(uint64_t* p, uint64_t n, uint64_t v) {
    const uint64_t pairs = n >> 1;
    ulonglong2* q = reinterpret_cast<ulonglong2*>(p);
    const ulonglong2 vv = make_ulonglong2(v, v);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < pairs;
         i += (uint64_t)gridDim.x * blockDim.x)
        q[i] = vv;
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[n - 1] = v;
}
// The same with nontemporal stores, for sets far larger than the caches: the cleared
// lines are not kept dirty in L2 / MALL ahead of the stage that scatters into the set
// (measured: the backward stage and the meet run faster after it).
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
__global__ void k_fill16nt(uint64_t* p, uint64_t n, uint64_t v) {
    const uint64_t pairs = n >> 1;
    u64x2* q = reinterpret_cast<u64x2*>(p);
    u64x2 vv;
    vv.x = v;
    vv.y = v;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < pairs;
         i += (uint64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(vv, &q[i]);
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[n - 1] = v;
}
constexpr uint64_t kFillNtWords = (64ull << 20) / 8;
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
    t_ev_used = false;
}

bool take_launch_events_used() {
    const bool used = t_ev_used;
    t_ev_used = false;
    t_ev_start = t_ev_stop = nullptr;
    return used;
}

hipError_t launch_fill(uint64_t* p, uint64_t n, uint64_t value, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (((uintptr_t)p & 15) == 0 && n >= kFillNtWords)
        hipLaunchKernelGGL(k_fill16nt, dim3(grid_for(n >> 1, kBlock, 16384)), dim3(kBlock), 0, st, p, n, value);
    else if (((uintptr_t)p & 15) == 0 && n >= 2)
        hipLaunchKernelGGL(k_fill16, dim3(grid_for(n >> 1, kBlock, 16384)), dim3(kBlock), 0, st, p, n, value);
    else
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, st, p, n, value);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Segment tables: the direction of orientation (ia, ie) is
// (cos el cos az, cos el sin az, sin el) with az = 2*pi*ia/na, el = 2*pi*ie/na; the
// segment end and the S sample points at fractions s/S of the length are rounded to
// the nearest voxel, halves away from zero (halves recognised within 1e-9, so that
// FP64 evaluation order cannot split an exact tie such as 25*cos 60 deg).
// ---------------------------------------------------------------------------
__device__ int round_voxel(double v) {
    double a = fabs(v);
    double f = floor(a);
    double frac = a - f;
    int r = (int)f + ((frac > 0.5 - 1e-9) ? 1 : 0);
    return v < 0 ? -r : r;
}

__global__ void k_tables(int na, int S, int L, short4* off, short4* sweep, unsigned int* maxn2) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= na * na) return;
    int ia = o / na, ie = o % na;
    double saz, caz, sel, cel;
    sincospi(2.0 * (double)ia / (double)na, &saz, &caz);
    sincospi(2.0 * (double)ie / (double)na, &sel, &cel);
    double dx = cel * caz, dy = cel * saz, dz = sel;
    int ex = round_voxel((double)L * dx), ey = round_voxel((double)L * dy), ez = round_voxel((double)L * dz);
    off[o] = make_short4((short)ex, (short)ey, (short)ez, 0);
    atomicMax(maxn2, (unsigned int)(ex * ex + ey * ey + ez * ez));
    for (int s = 1; s <= S; ++s) {
        double len = (double)(s * L) / (double)S;
        sweep[(size_t)o * S + (s - 1)] = make_short4((short)round_voxel(len * dx), (short)round_voxel(len * dy),
                                                     (short)round_voxel(len * dz), 0);
    }
}

hipError_t launch_tables(int na, int S, int L, short4* off, short4* sweep, unsigned int* maxn2,
                         hipStream_t st) {
    int cnt = na * na;
    hipLaunchKernelGGL(k_tables, dim3((cnt + 255) / 256), dim3(256), 0, st, na, S, L, off, sweep, maxn2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Raster: one thread per 64-voxel word.  For a row (y, z) a box dilated by r
// (Euclidean Minkowski sum) covers x in [lo_x - w, hi_x + w] with
// w = floor(sqrt(r^2 - dy^2 - dz^2)), dy/dz the distances of the row to the box's
// y/z ranges; a sphere of radius R dilated by r covers x in [cx - w, cx + w] with
// w = floor(sqrt((R+r)^2 - dy^2 - dz^2)).  Bits past the grid edge are set.
// ---------------------------------------------------------------------------
__device__ long long isqrt_floor(long long v) {
    long long s = (long long)sqrt((double)v);
    while (s > 0 && s * s > v) --s;
    while ((s + 1) * (s + 1) <= v) ++s;
    return s;
}

__device__ uint64_t span_bits(long long lo, long long hi, long long x0) {
    long long a = lo - x0, b = hi - x0;
    if (b < 0 || a > 63) return 0;
    if (a < 0) a = 0;
    if (b > 63) b = 63;
    uint64_t top = (b == 63) ? ~0ull : ((1ull << (b + 1)) - 1);
    uint64_t bot = (1ull << a) - 1;
    return top & ~bot;
}

constexpr int kObsChunk = 256;

__global__ void k_raster(uint64_t* occ, int n, int wpr, int r, const int32_t* boxes, int nbox,
                         const int32_t* spheres, int nsph, RasterInline inl, int use_inl) {
    // obstacle lists (in the kernel arguments, or in memory, possibly mapped host memory)
    // are staged through LDS in chunks
    __shared__ int32_t sb[kObsChunk * 6];
    __shared__ int32_t ss[kObsChunk * 4];
    const uint64_t total = (uint64_t)n * n * wpr;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < total; base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = base + threadIdx.x;
        const bool live = i < total;
        int xw = 0, y = 0, z = 0;
        if (live) {
            xw = (int)(i % wpr);
            uint64_t row = i / wpr;
            y = (int)(row % n);
            z = (int)(row / n);
        }
        const long long x0 = 64ll * xw;
        uint64_t bits = 0;
        for (int b0 = 0; b0 < nbox; b0 += kObsChunk) {
            const int cnt = min(kObsChunk, nbox - b0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt * 6; t += blockDim.x)
                sb[t] = use_inl ? inl.v[b0 * 6 + t] : boxes[b0 * 6 + t];
            __syncthreads();
            if (!live) continue;
            for (int b = 0; b < cnt; ++b) {
                const int32_t* B = sb + 6 * b;
                long long ylo = B[1], yhi = (long long)B[1] + B[4] - 1;
                long long zlo = B[2], zhi = (long long)B[2] + B[5] - 1;
                long long dy = y < ylo ? ylo - y : (y > yhi ? y - yhi : 0);
                long long dz = z < zlo ? zlo - z : (z > zhi ? z - zhi : 0);
                long long rem = (long long)r * r - dy * dy - dz * dz;
                if (rem < 0) continue;
                long long w = isqrt_floor(rem);
                bits |= span_bits((long long)B[0] - w, (long long)B[0] + B[3] - 1 + w, x0);
            }
        }
        for (int s0 = 0; s0 < nsph; s0 += kObsChunk) {
            const int cnt = min(kObsChunk, nsph - s0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt * 4; t += blockDim.x)
                ss[t] = use_inl ? inl.v[nbox * 6 + s0 * 4 + t] : spheres[s0 * 4 + t];
            __syncthreads();
            if (!live) continue;
            for (int b = 0; b < cnt; ++b) {
                const int32_t* P = ss + 4 * b;
                long long dy = y - P[1], dz = z - P[2];
                long long rr = (long long)P[3] + r;
                long long rem = rr * rr - dy * dy - dz * dz;
                if (rem < 0) continue;
                long long w = isqrt_floor(rem);
                bits |= span_bits((long long)P[0] - w, (long long)P[0] + w, x0);
            }
        }
        if (!live) continue;
        if (x0 + 64 > n) bits |= span_bits(n, x0 + 63, x0);
        occ[i] = bits;
    }
}

hipError_t launch_raster(uint64_t* occ, int n, int wpr, int r, const int32_t* boxes, int nbox,
                         const int32_t* spheres, int nsph, hipStream_t st) {
    uint64_t total = (uint64_t)n * n * wpr;
    RasterInline none{};
    hipLaunchKernelGGL(k_raster, dim3(grid_for(total)), dim3(kBlock), 0, st, occ, n, wpr, r, boxes, nbox,
                       spheres, nsph, none, 0);
    return hipGetLastError();
}

hipError_t launch_raster_inline(uint64_t* occ, int n, int wpr, int r, const RasterInline& inl, int nbox, int nsph,
                                hipStream_t st) {
    if (nbox < 0 || nsph < 0 || (int64_t)nbox * 6 + (int64_t)nsph * 4 > kRasterInline) return hipErrorInvalidValue;
    uint64_t total = (uint64_t)n * n * wpr;
    hipLaunchKernelGGL(k_raster, dim3(grid_for(total)), dim3(kBlock), 0, st, occ, n, wpr, r, (const int32_t*)nullptr,
                       nbox, (const int32_t*)nullptr, nsph, inl, 1);
    return hipGetLastError();
}

// Grid of one tick with moving boxes ("Dynamic Obstacles"): dst = src OR the boxes of
// `db` dilated by r, word by word (the same row spans as k_raster).  src is the static
// grid (its bits past the grid edge are already set), or dst itself when a further
// launch adds more boxes.  The boxes travel in the kernel arguments, so the call needs
// no staging memory.
__global__ void k_raster_dyn(uint64_t* dst, const uint64_t* src, int n, int wpr, int r, DynBoxes db) {
    const uint64_t total = (uint64_t)n * n * wpr;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int xw = (int)(i % wpr);
        const uint64_t row = i / wpr;
        const long long y = (long long)(row % n), z = (long long)(row / n);
        const long long x0 = 64ll * xw;
        uint64_t bits = src[i];
        for (int b = 0; b < db.count; ++b) {
            const int32_t* B = db.b + 6 * b;
            const long long ylo = B[1], yhi = (long long)B[1] + B[4] - 1;
            const long long zlo = B[2], zhi = (long long)B[2] + B[5] - 1;
            const long long dy = y < ylo ? ylo - y : (y > yhi ? y - yhi : 0);
            const long long dz = z < zlo ? zlo - z : (z > zhi ? z - zhi : 0);
            const long long rem = (long long)r * r - dy * dy - dz * dz;
            if (rem < 0) continue;
            const long long w = isqrt_floor(rem);
            bits |= span_bits((long long)B[0] - w, (long long)B[0] + B[3] - 1 + w, x0);
        }
        dst[i] = bits;
    }
}

hipError_t launch_raster_dyn(uint64_t* dst, const uint64_t* src, int n, int wpr, int r, const DynBoxes& db,
                             hipStream_t st) {
    const uint64_t total = (uint64_t)n * n * wpr;
    hipLaunchKernelGGL(k_raster_dyn, dim3(grid_for(total)), dim3(kBlock), 0, st, dst, src, n, wpr, r, db);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Orientation reachability O_k (k = 0..n): orientations the chain can have after k
// joints, positions ignored.  Yaw joints move only the azimuth index and pitch joints
// only the elevation index, so O_k = IA_k x IE_k with IA_k (IE_k) the start index
// plus the cyclic Minkowski sum of the yaw (pitch) windows so far.  One block;
// written as 256-bit rows: rows_ie[(k*na + ia)*4 + w] holds bit ie,
// rows_ia[(k*na + ie)*4 + w] holds bit ia.
// ---------------------------------------------------------------------------
__global__ void k_orient(OrientArgs oa, uint64_t* rows_ie, uint64_t* rows_ia) {
    const int n = oa.n, na = oa.na, ia0 = oa.ia0, ie0 = oa.ie0;
    __shared__ uint8_t A[kMaxNa], E[kMaxNa], T[kMaxNa];
    __shared__ uint64_t Abits[4], Ebits[4];
    const int tid = threadIdx.x;
    for (int t = tid; t < na; t += blockDim.x) {
        A[t] = (t == ia0);
        E[t] = (t == ie0);
    }
    if (tid < 4) {
        Abits[tid] = (ia0 >> 6) == tid ? 1ull << (ia0 & 63) : 0ull;
        Ebits[tid] = (ie0 >> 6) == tid ? 1ull << (ie0 & 63) : 0ull;
    }
    __syncthreads();
    for (int k = 0; k <= n; ++k) {
        if (k > 0) {
            const bool yaw = oa.type[k - 1] == 0;
            const int lo = oa.lo[k - 1], hi = oa.hi[k - 1];
            uint8_t* S = yaw ? A : E;
            const uint64_t* Sb = yaw ? Abits : Ebits;     // S as bits (gathered below for k - 1)
            // t is reached iff S holds a value in the circular interval t - hi .. t - lo:
            // one masked AND of the bit rows per value (no loop over the window)
            for (int t = tid; t < na; t += blockDim.x) {
                uint64_t m[4] = {0, 0, 0, 0};
                if (hi - lo + 1 >= na) {
                    mask_range(m, 0, na - 1);
                } else {
                    const int s0 = wrap_na(t - hi, na), e0 = s0 + (hi - lo);
                    if (e0 < na) {
                        mask_range(m, s0, e0);
                    } else {
                        mask_range(m, s0, na - 1);
                        mask_range(m, 0, e0 - na);
                    }
                }
                T[t] = ((m[0] & Sb[0]) | (m[1] & Sb[1]) | (m[2] & Sb[2]) | (m[3] & Sb[3])) != 0;
            }
            __syncthreads();
            for (int t = tid; t < na; t += blockDim.x) S[t] = T[t];
            __syncthreads();
        }
        {
            // one ballot per wave gathers 64 bits of each set (256 threads cover na <= 256)
            const bool a = tid < na && A[tid];
            const bool e = tid < na && E[tid];
            const unsigned long long ab = __ballot(a);
            const unsigned long long eb = __ballot(e);
            if ((tid & 63) == 0) {
                Abits[tid >> 6] = ab;
                Ebits[tid >> 6] = eb;
            }
        }
        __syncthreads();
        for (int idx = tid; idx < na * 4; idx += blockDim.x) {
            int v = idx >> 2, w = idx & 3;
            rows_ie[((size_t)k * na + v) * 4 + w] = A[v] ? Ebits[w] : 0ull;
            rows_ia[((size_t)k * na + v) * 4 + w] = E[v] ? Abits[w] : 0ull;
        }
        __syncthreads();
    }
}

hipError_t launch_orient(const OrientArgs& a, uint64_t* rows_ie, uint64_t* rows_ia, hipStream_t st) {
    hipLaunchKernelGGL(k_orient, dim3(1), dim3(256), 0, st, a, rows_ie, rows_ia);
    return hipGetLastError();
}

// Copies counters into mapped host memory, then (system-scope fence first) writes the
// sequence number `seq` to `flag`, which the host polls instead of synchronising the
// stream.
__global__ void k_publish(const unsigned long long* src, unsigned long long* dst, int n, unsigned long long* flag,
                          unsigned long long seq) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0 && flag) {
        __threadfence_system();
        __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

hipError_t launch_publish(const unsigned long long* src, unsigned long long* dst, int n, unsigned long long* flag,
                          unsigned long long seq, hipStream_t st) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, st, src, dst, n, flag, seq);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Seeds: F_0 = {(base, o0)} if the base is free; B_n = {(target, o) : o in O_n} if
// the target is free.
// ---------------------------------------------------------------------------
// The seeds also write their state lists (so that the first stages need no compaction).
__global__ void k_seed_fwd(SetView s, GridView g, int x, int y, int z, int ia, int ie, uint64_t* list,
                           unsigned long long* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && cell_free(g, x, y, z)) {
        if (set_insert(s, x, y, z, ia, ie) > 0) {
            list[0] = pack_key(x, y, z, ia, ie);
            atomicAdd(counter, 1ull);
        }
    }
}

// rows_ie: reachable final orientations (used when prune); cone: the approach cone's
// final orientations (null: no cone); both as [ia][4 words of ie bits].
__global__ void k_seed_bwd(SetView s, GridView g, int x, int y, int z, const uint64_t* rows_ie, int prune,
                           const uint64_t* cone, uint64_t* list, unsigned long long* counter) {
    const int na = s.na;
    const bool free_cell = cell_free(g, x, y, z);
    const int lane = threadIdx.x & 63;
    // a wave-uniform loop: every lane takes part in the ballot that places the keys
    for (int o0 = (blockIdx.x * blockDim.x + threadIdx.x) & ~63; o0 < na * na; o0 += gridDim.x * blockDim.x) {
        const int o = o0 + lane;
        bool ok = false;
        int ia = 0, ie = 0;
        if (free_cell && o < na * na) {
            ia = o / na;
            ie = o % na;
            ok = !prune || ((rows_ie[ia * 4 + (ie >> 6)] >> (ie & 63)) & 1ull);
            ok = ok && (!cone || ((cone[ia * 4 + (ie >> 6)] >> (ie & 63)) & 1ull));
        }
        // a dense set whose orientation index is ia * na + ie, with word-aligned voxel
        // blocks: the wave's 64 orientations are the 64 bits of one word, set by one atomic
        uint64_t bit0 = 0;
        const bool one_word = s.kind == kDense && !s.fast_ia && ((na * na) & 63) == 0 &&
                              dense_bit(s, x, y, z, o0 / na, o0 % na, bit0) && (bit0 & 63) == 0;
        if (one_word) {
            const uint64_t want = __ballot(ok);
            uint64_t added = 0;
            if (lane == 0 && want)
                added = want & ~(uint64_t)atomicOr((unsigned long long*)&s.words[bit0 >> 6], (unsigned long long)want);
            added = __shfl(added, 0, 64);
            ok = (added >> lane) & 1ull;
        } else {
            ok = ok && set_insert(s, x, y, z, ia, ie) > 0;
        }
        const uint64_t bal = __ballot(ok);
        unsigned long long base = 0;
        if (lane == 0 && bal) base = atomicAdd(counter, (unsigned long long)__popcll(bal));
        base = __shfl(base, 0, 64);
        if (ok) list[base + __popcll(bal & ((1ull << lane) - 1))] = pack_key(x, y, z, ia, ie);
    }
}

hipError_t launch_seed_fwd(SetView s, GridView g, int x, int y, int z, int ia, int ie, uint64_t* list,
                           unsigned long long* counter, hipStream_t st) {
    hipLaunchKernelGGL(k_seed_fwd, dim3(1), dim3(64), 0, st, s, g, x, y, z, ia, ie, list, counter);
    return hipGetLastError();
}

hipError_t launch_seed_bwd(SetView s, GridView g, int x, int y, int z, const uint64_t* rows_ie, int prune,
                           const uint64_t* cone, uint64_t* list, unsigned long long* counter, hipStream_t st) {
    hipLaunchKernelGGL(k_seed_bwd, dim3(grid_for((uint64_t)s.na * s.na)), dim3(kBlock), 0, st, s, g, x, y, z,
                       rows_ie, prune, cone, list, counter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward stage (Steps 1 and 2A): every state of the input list is tried against
// every angle of the joint window; the successor is kept if it lies within the
// forward pruning radius of the target (eqs 5-6) and the new segment is clear.
// One work item per (state, angle).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_expand_fwd(const uint64_t* __restrict__ in, uint64_t count,
                                                       SetView out, GridView g, JointView j, int tx, int ty,
                                                       int tz, long long r2, unsigned long long* counter,
                                                       unsigned long long* overflow) {
    const int na = out.na;
    const uint32_t nA = (uint32_t)(j.hi - j.lo + 1);
    unsigned long long added = 0, ovf = 0;
    // Work item idx = i * nA + ai walks the grid stride as (state, angle) pairs: one
    // 64-bit division per thread, none per item.
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t idx0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t si = stride / nA;
    const uint32_t sa = (uint32_t)(stride - si * nA);
    uint64_t i = idx0 / nA;
    uint32_t ai = (uint32_t)(idx0 - i * nA);
    for (; i < count; i += si, ai += sa, i += (ai >= nA) ? 1 : 0, ai -= (ai >= nA) ? nA : 0) {
        int a = j.lo + (int)ai;
        int x, y, z, ia, ie;
        unpack_key(in[i], x, y, z, ia, ie);
        if (ia >= na || ie >= na) continue;
        if (j.type == 0)
            ia = wrap_na(ia + a, na);
        else
            ie = wrap_na(ie + a, na);
        const int o = ia * na + ie;
        const short4 d = j.off[o];
        const int x2 = x + d.x, y2 = y + d.y, z2 = z + d.z;
        if (r2 >= 0) {
            long long ex = x2 - tx, ey = y2 - ty, ez = z2 - tz;
            if (ex * ex + ey * ey + ez * ez > r2) continue;
        }
        if (!segment_clear_all(g, j, o, x, y, z)) continue;
        int r = set_insert(out, x2, y2, z2, ia, ie);
        if (r > 0)
            ++added;
        else if (r < 0)
            ++ovf;
    }
    block_add(added, counter);
    if (ovf) atomicAdd(overflow, ovf);
}

hipError_t launch_expand_fwd(const uint64_t* in, uint64_t count, SetView out, GridView g, JointView j,
                             int tx, int ty, int tz, long long r2, unsigned long long* counter,
                             unsigned long long* overflow, hipStream_t st, Shape sh) {
    uint64_t work = count * (uint64_t)(j.hi - j.lo + 1);
    if (work == 0) return hipSuccess;
    launch_timed(k_expand_fwd, dim3(grid_for(work, kBlock, sh.max_blocks)), dim3(kBlock), 0, st, in, count,
                       out, g, j, tx, ty, tz, r2, counter, overflow);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Backward stage: for a state (p', o') after segment k, the start p = p' - off[o']
// of segment k is the same for every angle of joint k, so the clearance of the
// segment is tested once; the predecessors are (p, o' turned back by a) for every
// a in the window, a cyclic run along the joint's axis, filtered by O_{k-1} and the
// backward pruning radius around the base (eqs 7-8).  This kernel serves dense
// outputs whose fastest orientation axis is the joint's axis: the run is set with at
// most a few masked atomicOr (other outputs: k_expand_bwd_set).
// ---------------------------------------------------------------------------
template <int NP, bool COUNT>
__global__ void __launch_bounds__(kBlock) k_expand_bwd(const uint64_t* __restrict__ in, uint64_t count,
                                                       SetView out, GridView g, JointView j, int bx, int by,
                                                       int bz, long long r2, const uint64_t* __restrict__ orows,
                                                       unsigned long long* counter,
                                                       unsigned long long* overflow) {
    const int na = out.na;
    const int nA = j.hi - j.lo + 1;
    const bool yaw = j.type == 0;
    unsigned long long added = 0, ovf = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int x2, y2, z2, ia2, ie2;
        unpack_key(in[i], x2, y2, z2, ia2, ie2);
        if (ia2 >= na || ie2 >= na) continue;
        const int o2 = ia2 * na + ie2;
        const short4 d = j.off[o2];
        const int x = x2 - d.x, y = y2 - d.y, z = z2 - d.z;
        if (!cell_free(g, x, y, z)) continue;
        if (r2 >= 0) {
            long long ex = x - bx, ey = y - by, ez = z - bz;
            if (ex * ex + ey * ey + ez * ez > r2) continue;
        }
        if (!segment_clear_all(g, j, o2, x, y, z)) continue;
        const int v = yaw ? ia2 : ie2;
        const int other = yaw ? ie2 : ia2;
        uint64_t m[4] = {0, 0, 0, 0};
        if (nA >= na) {
            mask_range(m, 0, na - 1);
        } else {
            int s = wrap_na(v - j.hi, na);
            int e = s + nA - 1;
            if (e < na) {
                mask_range(m, s, e);
            } else {
                mask_range(m, s, na - 1);
                mask_range(m, 0, e - na);
            }
        }
        if (orows) {
            const uint64_t* row = orows + (size_t)other * 4;
            for (int w = 0; w < 4; ++w) m[w] &= row[w];
        }
        uint64_t bit0;
        if (!dense_bit(out, x, y, z, yaw ? 0 : ia2, yaw ? ie2 : 0, bit0)) {
            ++ovf;
            continue;
        }
        // the run as (up to) five word-aligned parts: all atomics are issued before any
        // result is used, so that they are in flight together
        const uint64_t word0 = bit0 >> 6;
        const int sh = (int)(bit0 & 63);
        uint64_t part[5];
#pragma unroll
        for (int w = 0; w < 5; ++w) {
            const uint64_t cur = w < 4 ? m[w] : 0ull;
            const uint64_t prev = w > 0 ? m[w - 1] : 0ull;
            part[w] = (cur << sh) | (sh ? prev >> (64 - sh) : 0ull);
        }
        // a row of na bits spans at most NP words (NP is fixed per launch from na); only
        // non-empty parts are sent, and all of them are in flight before the first result
        // is used (the empty asm statements keep the uses out of the conditional sends)
        if constexpr (COUNT) {
            uint64_t old[NP];
#pragma unroll
            for (int w = 0; w < NP; ++w) {
                old[w] = ~0ull;
                if (part[w])
                    old[w] = atomicOr((unsigned long long*)&out.words[word0 + w], (unsigned long long)part[w]);
            }
#pragma unroll
            for (int w = 0; w < NP; ++w) asm volatile("" : "+v"(old[w]));
#pragma unroll
            for (int w = 0; w < NP; ++w) added += __popcll(part[w] & ~old[w]);
        } else {
            // no count wanted: the atomics return nothing and the wave does not wait
#pragma unroll
            for (int w = 0; w < NP; ++w)
                if (part[w]) atomicOr((unsigned long long*)&out.words[word0 + w], (unsigned long long)part[w]);
        }
    }
    if constexpr (COUNT) block_add(added, counter);
    if (ovf) atomicAdd(overflow, ovf);
}

// The same stage into a hash set (or a dense set whose fast axis is not the joint's):
// the predecessor run is inserted one orientation per lane, a group of lanes per state.
__global__ void __launch_bounds__(kBlock) k_expand_bwd_set(const uint64_t* __restrict__ in, uint64_t count,
                                                           SetView out, GridView g, JointView j, int bx, int by,
                                                           int bz, long long r2, const uint64_t* __restrict__ orows,
                                                           unsigned long long* counter,
                                                           unsigned long long* overflow, int lg) {
    const int na = out.na;
    const bool yaw = j.type == 0;
    const int G = 1 << lg;
    const int lane = threadIdx.x & 63, sub = lane & (G - 1), grp = lane >> lg;
    const uint64_t per_wave = 64u >> lg;
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long added = 0, ovf = 0;
    for (uint64_t base = wave * per_wave; base < count; base += nwaves * per_wave) {
        const uint64_t i = base + (uint64_t)grp;
        if (i >= count) continue;
        int x2, y2, z2, ia2, ie2;
        unpack_key(in[i], x2, y2, z2, ia2, ie2);
        if (ia2 >= na || ie2 >= na) continue;
        const int o2 = ia2 * na + ie2;
        const short4 d = j.off[o2];
        const int x = x2 - d.x, y = y2 - d.y, z = z2 - d.z;
        if (!cell_free(g, x, y, z)) continue;
        if (r2 >= 0) {
            long long ex = x - bx, ey = y - by, ez = z - bz;
            if (ex * ex + ey * ey + ez * ez > r2) continue;
        }
        if (!segment_clear_all(g, j, o2, x, y, z)) continue;
        const int v = yaw ? ia2 : ie2;
        const uint64_t* row = orows ? orows + (size_t)(yaw ? ie2 : ia2) * 4 : nullptr;
        for (int a = j.lo + sub; a <= j.hi; a += G) {
            const int u = wrap_na(v - a, na);
            if (row && !((row[u >> 6] >> (u & 63)) & 1ull)) continue;
            int r = set_insert(out, x, y, z, yaw ? u : ia2, yaw ? ie2 : u);
            if (r > 0)
                ++added;
            else if (r < 0)
                ++ovf;
        }
    }
    block_add(added, counter);
    if (ovf) atomicAdd(overflow, ovf);
}

// Clearing of a dense set built by k_expand_bwd from the list `in`: for every input
// state, the whole orientation row of its predecessor voxel that the stage may have
// touched is set to zero (tests skipped: a superset of the written words, all inside
// the set), so the set is all zero afterwards without a pass over all of its words.
__global__ void __launch_bounds__(kBlock) k_unexpand_bwd(const uint64_t* __restrict__ in, uint64_t count,
                                                         SetView out, JointView j) {
    const int na = out.na;
    const bool yaw = j.type == 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int x2, y2, z2, ia2, ie2;
        unpack_key(in[i], x2, y2, z2, ia2, ie2);
        if (ia2 >= na || ie2 >= na) continue;
        const short4 d = j.off[ia2 * na + ie2];
        uint64_t bit0;
        if (!dense_bit(out, x2 - d.x, y2 - d.y, z2 - d.z, yaw ? 0 : ia2, yaw ? ie2 : 0, bit0)) continue;
        const uint64_t w1 = (bit0 + (uint64_t)na - 1) >> 6;
        for (uint64_t w = bit0 >> 6; w <= w1; ++w) out.words[w] = 0;
    }
}

// Clearing of a dense set by its own member list: the word of every listed state is set
// to zero (the list holds every member the set ever had: members are only removed after
// it was made).
__global__ void __launch_bounds__(kBlock) k_unlist(const uint64_t* __restrict__ list, uint64_t count, SetView s) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int x, y, z, ia, ie;
        unpack_key(list[i], x, y, z, ia, ie);
        uint64_t bit;
        if (ia < s.na && ie < s.na && dense_bit(s, x, y, z, ia, ie, bit)) s.words[bit >> 6] = 0;
    }
}

hipError_t launch_unlist(const uint64_t* list, uint64_t count, SetView s, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unlist, dim3(grid_for(count, kBlock, 16384)), dim3(kBlock), 0, st, list, count, s);
    return hipGetLastError();
}

hipError_t launch_unexpand_bwd(const uint64_t* in, uint64_t count, SetView out, JointView j, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unexpand_bwd, dim3(grid_for(count, kBlock, 16384)), dim3(kBlock), 0, st, in, count, out, j);
    return hipGetLastError();
}

template <bool COUNT>
void launch_bwd_dense(int np, dim3 grid, hipStream_t st, const uint64_t* in, uint64_t count, SetView out,
                      GridView g, JointView j, int bx, int by, int bz, long long r2, const uint64_t* orows,
                      unsigned long long* counter, unsigned long long* overflow) {
    if (np == 2)
        launch_timed(k_expand_bwd<2, COUNT>, grid, dim3(kBlock), 0, st, in, count, out, g, j, bx, by, bz, r2,
                           orows, counter, overflow);
    else if (np == 3)
        launch_timed(k_expand_bwd<3, COUNT>, grid, dim3(kBlock), 0, st, in, count, out, g, j, bx, by, bz, r2,
                           orows, counter, overflow);
    else if (np == 4)
        launch_timed(k_expand_bwd<4, COUNT>, grid, dim3(kBlock), 0, st, in, count, out, g, j, bx, by, bz, r2,
                           orows, counter, overflow);
    else
        launch_timed(k_expand_bwd<5, COUNT>, grid, dim3(kBlock), 0, st, in, count, out, g, j, bx, by, bz, r2,
                           orows, counter, overflow);
}

hipError_t launch_expand_bwd(const uint64_t* in, uint64_t count, SetView out, GridView g, JointView j,
                             int bx, int by, int bz, long long r2, const uint64_t* orows,
                             unsigned long long* counter, unsigned long long* overflow, hipStream_t st, Shape sh) {
    if (count == 0) return hipSuccess;
    const bool run_dense = out.kind == kDense && ((out.fast_ia != 0) == (j.type == 0));
    if (run_dense) {
        const int np = ((out.na + 63) >> 6) + 1;   // words a row of na bits can touch
        const dim3 grid(grid_for(count, kBlock, sh.max_blocks));
        if (counter)
            launch_bwd_dense<true>(np, grid, st, in, count, out, g, j, bx, by, bz, r2, orows, counter, overflow);
        else
            launch_bwd_dense<false>(np, grid, st, in, count, out, g, j, bx, by, bz, r2, orows, counter, overflow);
    } else {
        const int lg = std::clamp(group_log2_for(count, j.hi - j.lo + 1) + sh.lg_bias, 0, 6);
        launch_timed(k_expand_bwd_set, dim3(grid_for(count << lg, kBlock, sh.max_blocks)), dim3(kBlock), 0, st,
                           in, count, out, g, j, bx, by, bz, r2, orows, counter, overflow, lg);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compaction: the members of a set into a list.  A block takes tiles of
// kBlock * kCompactWords words (each thread keeps its words in registers), counts
// their members (dense: set bits; hash: occupied, not removed slots), computes a
// block-wide exclusive scan and reserves the tile's output range with one atomicAdd.
// ---------------------------------------------------------------------------
constexpr int kCompactWords = 16;

// q = n / d, r = n % d for n < 2^53, via a double reciprocal and one correction step.
__device__ __forceinline__ void divmod_big(uint64_t n, uint32_t d, double inv, uint64_t& q, uint32_t& r) {
    uint64_t qq = (uint64_t)((double)n * inv);
    int64_t rr = (int64_t)(n - qq * (uint64_t)d);
    while (rr < 0) {
        --qq;
        rr += d;
    }
    while (rr >= (int64_t)d) {
        ++qq;
        rr -= d;
    }
    q = qq;
    r = (uint32_t)rr;
}

// Position of the r-th set bit (r < popcount) of w, by popcount bisection.
__device__ __forceinline__ int select_bit(uint64_t w, unsigned int r) {
    int pos = 0;
    unsigned int c = (unsigned int)__popc((uint32_t)w);
    if (r >= c) {
        r -= c;
        w >>= 32;
        pos = 32;
    }
    uint32_t x = (uint32_t)w;
    c = (unsigned int)__popc(x & 0xffffu);
    if (r >= c) {
        r -= c;
        x >>= 16;
        pos += 16;
    }
    c = (unsigned int)__popc(x & 0xffu);
    if (r >= c) {
        r -= c;
        x >>= 8;
        pos += 8;
    }
    c = (unsigned int)__popc(x & 0xfu);
    if (r >= c) {
        r -= c;
        x >>= 4;
        pos += 4;
    }
    c = (unsigned int)__popc(x & 0x3u);
    if (r >= c) {
        r -= c;
        x >>= 2;
        pos += 2;
    }
    if (r >= (x & 1u)) pos += 1;
    return pos;
}

__device__ __forceinline__ int member_count(const SetView& s, uint64_t w) {
    if (s.kind == kDense) return __popcll(w);
    return (w != kEmpty && !(w & kDead)) ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_compact(SetView s, uint64_t* list, uint64_t cap,
                                                    unsigned long long* counter,
                                                    unsigned long long* overflow) {
    __shared__ unsigned int wave_off[kBlock / 64];
    __shared__ unsigned long long tile_base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t na2 = (uint32_t)(s.na * s.na);
    const double inv_na2 = 1.0 / (double)na2;
    const float inv_na = 1.0f / (float)s.na;
    const uint64_t tile = (uint64_t)kBlock * kCompactWords;
    for (uint64_t t0 = blockIdx.x * tile; t0 < s.cap; t0 += (uint64_t)gridDim.x * tile) {
        uint64_t wv[kCompactWords];
        unsigned int c = 0;
#pragma unroll
        for (int j = 0; j < kCompactWords; ++j) {
            uint64_t i = t0 + (uint64_t)j * kBlock + tid;
            wv[j] = i < s.cap ? s.words[i] : (s.kind == kDense ? 0ull : kEmpty);
            c += member_count(s, wv[j]);
        }
        unsigned int incl = c;
        for (int off = 1; off < 64; off <<= 1) {
            unsigned int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        if (lane == 63) wave_off[wave] = incl;
        __syncthreads();
        if (tid == 0) {
            unsigned int tot = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                unsigned int v = wave_off[w];
                wave_off[w] = tot;
                tot += v;
            }
            tile_base = tot ? atomicAdd(counter, (unsigned long long)tot) : 0ull;
        }
        __syncthreads();
        if (s.kind == kDense) {
            // Wave-balanced emission.  Round j covers the wave's 64 consecutive words;
            // lane t of the round emits states t, t + 64, ... of the round, finding its
            // word by bisection over the lanes' prefix counts and its bit by popcount
            // bisection, so a few dense words do not serialise the wave.
            uint64_t out = tile_base + wave_off[wave];
            const uint32_t nx = (uint32_t)s.nx, ny = (uint32_t)s.ny;
#pragma unroll
            for (int j = 0; j < kCompactWords; ++j) {
                const uint64_t w = wv[j];
                if (__ballot(w != 0) == 0) continue;   // nothing in this round
                const unsigned int cj = (unsigned int)__popcll(w);
                unsigned int ij = cj;
                for (int off = 1; off < 64; off <<= 1) {
                    const unsigned int t = __shfl_up(ij, off, 64);
                    if (lane >= off) ij += t;
                }
                const unsigned int T = __shfl(ij, 63, 64);
                if (T == 0) continue;
                const unsigned int ex = ij - cj;
                const uint64_t i = t0 + (uint64_t)j * kBlock + tid;
                uint64_t vox;
                uint32_t o0;
                divmod_big(i * 64, na2, inv_na2, vox, o0);
                const uint32_t v32 = (uint32_t)vox;
                const uint32_t rest = v32 / nx;
                const uint32_t dx0 = v32 - rest * nx, dy0 = rest % ny, dz0 = rest / ny;
                const unsigned int rounds = (T + 63u) & ~63u;
                for (unsigned int t = (unsigned int)lane; t < rounds; t += 64) {
                    int L = 0;
                    for (int step = 32; step > 0; step >>= 1) {
                        const unsigned int e = __shfl(ex, L + step, 64);
                        if (e <= t) L += step;
                    }
                    const uint64_t wl = __shfl(w, L, 64);
                    const unsigned int r = t - __shfl(ex, L, 64);
                    const int ol = __shfl((int)o0, L, 64);
                    uint32_t dx = __shfl(dx0, L, 64), dy = __shfl(dy0, L, 64), dz = __shfl(dz0, L, 64);
                    if (t >= T) continue;
                    int o = ol + select_bit(wl, r);
                    while (o >= (int)na2) {
                        o -= (int)na2;
                        if (++dx == nx) {
                            dx = 0;
                            if (++dy == ny) {
                                dy = 0;
                                ++dz;
                            }
                        }
                    }
                    // o / na by a float reciprocal (o < 2^16), corrected to the exact quotient
                    int hi = (int)((float)o * inv_na);
                    hi -= hi * s.na > o ? 1 : 0;
                    hi += (hi + 1) * s.na <= o ? 1 : 0;
                    const int lo = o - hi * s.na;
                    const int ia = s.fast_ia ? lo : hi;
                    const int ie = s.fast_ia ? hi : lo;
                    const uint64_t p = out + t;
                    if (p < cap)
                        list[p] = pack_key(s.x0 + (int)dx, s.y0 + (int)dy, s.z0 + (int)dz, ia, ie);
                    else
                        atomicAdd(overflow, 1ull);
                }
                out += T;
            }
        } else if (c) {
            uint64_t pos = tile_base + wave_off[wave] + (incl - c);
#pragma unroll
            for (int j = 0; j < kCompactWords; ++j) {
                const uint64_t w = wv[j];
                if (member_count(s, w)) {
                    if (pos < cap)
                        list[pos] = w;
                    else
                        atomicAdd(overflow, 1ull);
                    ++pos;
                }
            }
        }
        __syncthreads();
    }
}

// Measurement: non-zero words of a set's structure (one grid-stride pass).
__global__ void __launch_bounds__(kBlock) k_count_words(SetView s, unsigned long long* counter) {
    unsigned long long n = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < s.cap; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t w = s.words[i];
        n += s.kind == kDense ? (w != 0) : (w != kEmpty && !(w & kDead));
    }
    block_add(n, counter);
}

hipError_t launch_count_words(SetView s, unsigned long long* counter, hipStream_t st) {
    if (s.cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_words, dim3(grid_for(s.cap, kBlock, 8192)), dim3(kBlock), 0, st, s, counter);
    return hipGetLastError();
}

hipError_t launch_compact(SetView s, uint64_t* list, uint64_t cap, unsigned long long* counter,
                          unsigned long long* overflow, hipStream_t st) {
    uint64_t tiles = (s.cap + (uint64_t)kBlock * kCompactWords - 1) / ((uint64_t)kBlock * kCompactWords);
    uint32_t blocks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(tiles, 1), 4096);
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(kBlock), 0, st, s, list, cap, counter, overflow);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Join: C_m = F_m intersected with B_m, in place in F_m's structure; counts |C_m|.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_join(const uint64_t* __restrict__ flist, uint64_t count, SetView f,
                                                 SetView b, unsigned long long* counter) {
    unsigned long long kept = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t key = flist[i];
        if (set_member(b, key))
            ++kept;
        else
            set_remove(f, key);
    }
    block_add(kept, counter);
}

hipError_t launch_join(const uint64_t* flist, uint64_t count, SetView f, SetView b,
                       unsigned long long* counter, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_join, dim3(grid_for(count)), dim3(kBlock), 0, st, flist, count, f, b, counter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Meet of the two pathways at the transition into stage m: every state of F_{m-1}
// is tried against every angle of joint m; a successor counts only if it is in B_m
// (tested first, before the segment test) and the segment is clear.  The hits are
// C_m = F_m intersected with B_m (inserted into `c`); the states of F_{m-1} without a
// hit are removed from `fprev`, which leaves D_{m-1}.  F_m is never built.  With
// Modes: kMeetInsert inserts the hits into `c` and marks D_{m-1}; kMeetCount only
// counts the hits (duplicates included), which sizes a hash C; kMeetMark only marks
// D_{m-1} (the canonical walk then steps into B_m: a successor of a D_{m-1} state
// with a clear segment that is in B_m is in C_m).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_meet(const uint64_t* __restrict__ flist, uint64_t count, SetView fprev,
                                                 SetView b, SetView c, GridView g, JointView j, int mode,
                                                 unsigned long long* c_count, unsigned long long* kept_count,
                                                 unsigned long long* overflow, int lg, int tx, int ty, int tz,
                                                 long long r2) {
    const int na = b.na;
    const int G = 1 << lg;
    const int lane = threadIdx.x & 63, sub = lane & (G - 1), grp = lane >> lg;
    const uint64_t per_wave = 64u >> lg;
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long added = 0, kept = 0, ovf = 0;
    for (uint64_t base = wave * per_wave; base < count; base += nwaves * per_wave) {
        const uint64_t i = base + (uint64_t)grp;
        uint64_t key = 0;
        int x = 0, y = 0, z = 0, ia = na, ie = na;
        bool hit = false;
        if (i < count) {
            key = flist[i];
            unpack_key(key, x, y, z, ia, ie);
        }
        const bool live = i < count && ia < na && ie < na;
        if (live) {
            for (int a = j.lo + sub; a <= j.hi; a += G) {
                int ia2 = ia, ie2 = ie;
                if (j.type == 0)
                    ia2 = wrap_na(ia + a, na);
                else
                    ie2 = wrap_na(ie + a, na);
                const int o = ia2 * na + ie2;
                const short4 d = j.off[o];
                const int x2 = x + d.x, y2 = y + d.y, z2 = z + d.z;
                if (r2 >= 0) {   // B_m lies in the forward pruning ball of stage m
                    const long long ex = x2 - tx, ey = y2 - ty, ez = z2 - tz;
                    if (ex * ex + ey * ey + ez * ez > r2) continue;
                }
                if (!set_member(b, pack_key(x2, y2, z2, ia2, ie2))) continue;
                if (!segment_clear_all(g, j, o, x, y, z)) continue;
                hit = true;
                if (mode != kMeetInsert) {
                    ++added;
                    if (mode == kMeetMark) break;   // one hit decides the state
                    continue;
                }
                int r = set_insert(c, x2, y2, z2, ia2, ie2);
                if (r > 0)
                    ++added;
                else if (r < 0)
                    ++ovf;
            }
        }
        // one decision per state: the OR of its group's hits
        const uint64_t bal = __ballot(hit);
        const uint64_t gm = lg == 6 ? bal : (bal >> (grp << lg)) & ((1ull << G) - 1);
        if (live && sub == 0) {
            if (gm)
                ++kept;
            else if (mode != kMeetCount)
                set_remove(fprev, key);
        }
    }
    block_add(added, c_count);
    block_add(kept, kept_count);
    if (ovf) atomicAdd(overflow, ovf);
}

hipError_t launch_meet(const uint64_t* flist, uint64_t count, SetView fprev, SetView b, SetView c, GridView g,
                       JointView j, int mode, unsigned long long* c_count, unsigned long long* kept_count,
                       unsigned long long* overflow, int tx, int ty, int tz, long long r2, hipStream_t st,
                       Shape sh) {
    if (count == 0) return hipSuccess;
    const int lg = std::clamp(group_log2_for(count, j.hi - j.lo + 1) + sh.lg_bias, 0, 6);
    hipLaunchKernelGGL(k_meet, dim3(grid_for(count << lg, kBlock, sh.max_blocks)), dim3(kBlock), 0, st, flist, count,
                       fprev, b, c, g, j, mode, c_count, kept_count, overflow, lg, tx, ty, tz, r2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// D_{k-1} = states of F_{k-1} with a clear move of joint k into D_k (already marked
// in fnext); the others are removed from fprev in place.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_dmark(const uint64_t* __restrict__ flist, uint64_t count,
                                                  SetView fprev, SetView fnext, GridView g, JointView j,
                                                  unsigned long long* counter, int lg, int tx, int ty, int tz,
                                                  long long r2) {
    const int na = fnext.na;
    const int G = 1 << lg;
    const int lane = threadIdx.x & 63, sub = lane & (G - 1), grp = lane >> lg;
    const uint64_t per_wave = 64u >> lg;
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long kept = 0;
    for (uint64_t base = wave * per_wave; base < count; base += nwaves * per_wave) {
        const uint64_t i = base + (uint64_t)grp;
        uint64_t key = 0;
        int x = 0, y = 0, z = 0, ia = na, ie = na;
        bool found = false;
        if (i < count) {
            key = flist[i];
            unpack_key(key, x, y, z, ia, ie);
        }
        const bool live = i < count && ia < na && ie < na;
        if (live) {
            for (int a = j.lo + sub; a <= j.hi && !found; a += G) {
                int ia2 = ia, ie2 = ie;
                if (j.type == 0)
                    ia2 = wrap_na(ia + a, na);
                else
                    ie2 = wrap_na(ie + a, na);
                const int o = ia2 * na + ie2;
                const short4 d = j.off[o];
                if (r2 >= 0) {   // F_k lies in the forward pruning ball of stage k
                    const long long ex = x + d.x - tx, ey = y + d.y - ty, ez = z + d.z - tz;
                    if (ex * ex + ey * ey + ez * ez > r2) continue;
                }
                if (!set_member(fnext, pack_key(x + d.x, y + d.y, z + d.z, ia2, ie2))) continue;
                if (!segment_clear_all(g, j, o, x, y, z)) continue;
                found = true;
            }
        }
        const uint64_t bal = __ballot(found);
        const uint64_t gm = lg == 6 ? bal : (bal >> (grp << lg)) & ((1ull << G) - 1);
        if (live && sub == 0) {
            if (gm)
                ++kept;
            else
                set_remove(fprev, key);
        }
    }
    block_add(kept, counter);
}

hipError_t launch_dmark(const uint64_t* flist, uint64_t count, SetView fprev, SetView fnext, GridView g,
                        JointView j, unsigned long long* counter, int tx, int ty, int tz, long long r2,
                        hipStream_t st, Shape sh) {
    if (count == 0) return hipSuccess;
    // at most 8 lanes per state: a lane tries several angles (measured faster than a
    // wave per state, whose lanes each try one)
    const int lg = std::clamp(std::min(group_log2_for(count, j.hi - j.lo + 1), 3) + sh.lg_bias, 0, 6);
    hipLaunchKernelGGL(k_dmark, dim3(grid_for(count << lg, kBlock, sh.max_blocks)), dim3(kBlock), 0, st, flist, count,
                       fprev, fnext, g, j, counter, lg, tx, ty, tz, r2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact end point ("Exact IK solution with discretized segment mappings"): the last two
// segments of a discrete pose, each with two DOF, are recomputed in FP64 so that the
// chain ends on the exact target.  P = end of the fixed first segments, J = the joint
// between the last two: |J - P| = L3, |T - J| = L4, in the plane of P, T and the
// discrete joint, on its side (the closing point nearest to it).  One thread per pose.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void unit_dir(double az, double el, double& x, double& y, double& z) {
    constexpr double kRad = 3.14159265358979323846 / 180.0;
    const double a = az * kRad, e = el * kRad;
    x = cos(e) * cos(a);
    y = cos(e) * sin(a);
    z = sin(e);
}

__device__ __forceinline__ double wrap180(double x) {
    double y = fmod(x, 360.0);
    if (y < 0.0) y += 360.0;
    return y > 180.0 ? y - 360.0 : y;
}

// (az, el) of s, as the name of its direction on the (az, el) torus -- (az, el) or
// (az + 180, 180 - el) -- nearer (raz, rel), unwrapped next to it; vertical s keeps raz
__device__ void angles_near(double sx, double sy, double sz, double raz, double rel, double& az, double& el) {
    constexpr double kDeg = 180.0 / 3.14159265358979323846;
    const double L = sqrt(sx * sx + sy * sy + sz * sz);
    const double e0 = asin(fmin(fmax(sz / L, -1.0), 1.0)) * kDeg;
    const double a0 = hypot(sx, sy) <= 1e-12 * L ? raz : atan2(sy, sx) * kDeg;
    const double da0 = wrap180(a0 - raz), de0 = wrap180(e0 - rel);
    const double da1 = wrap180(a0 + 180.0 - raz), de1 = wrap180(180.0 - e0 - rel);
    if (fabs(da1) + fabs(de1) < fabs(da0) + fabs(de0)) {
        az = raz + da1;
        el = rel + de1;
    } else {
        az = raz + da0;
        el = rel + de0;
    }
}

__global__ void __launch_bounds__(kBlock) k_refine(RefineArgs a, const int32_t* __restrict__ q,
                                                   const double* __restrict__ tgt, int64_t count,
                                                   double* __restrict__ out, int32_t* __restrict__ status) {
    const int n = a.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* qi = q + i * n;
        double* oi = out + i * n;
        double az = a.az0, el = a.el0;
        double px = a.base[0], py = a.base[1], pz = a.base[2];
        double paz = a.az0, pel = a.el0, az3 = 0, el3 = 0, az4 = 0, el4 = 0;
        for (int k = 0; k < n; ++k) {
            const double inc = (qi[k] / a.q_div) * a.step;
            oi[k] = inc;
            if (a.type[k] == 0)
                az += inc;
            else
                el += inc;
            if (k < n - 4) {
                double x, y, z;
                unit_dir(az, el, x, y, z);
                px = px + a.len[k] * x;
                py = py + a.len[k] * y;
                pz = pz + a.len[k] * z;
            }
            if (k == n - 5) {
                paz = az;
                pel = el;
            }
            if (k == n - 3) {
                az3 = az;
                el3 = el;
            }
            if (k == n - 1) {
                az4 = az;
                el4 = el;
            }
        }
        const double L3 = a.len[n - 3], L4 = a.len[n - 1];
        double jx, jy, jz;
        unit_dir(az3, el3, jx, jy, jz);
        jx = px + L3 * jx;
        jy = py + L3 * jy;
        jz = pz + L3 * jz;
        const double tx = tgt[i * 3], ty = tgt[i * 3 + 1], tz = tgt[i * 3 + 2];
        const double vx = tx - px, vy = ty - py, vz = tz - pz;
        const double d = sqrt(vx * vx + vy * vy + vz * vz);
        if (d == 0.0 || d > L3 + L4 || d < fabs(L3 - L4)) {
            status[i] = 1;
            continue;
        }
        const double ux = vx / d, uy = vy / d, uz = vz / d;
        const double aa = (L3 * L3 - L4 * L4 + d * d) / (2.0 * d);
        const double h = sqrt(fmax(L3 * L3 - aa * aa, 0.0));
        const double rx = jx - px, ry = jy - py, rz = jz - pz;
        const double ru = rx * ux + ry * uy + rz * uz;
        double wx = rx - ru * ux, wy = ry - ru * uy, wz = rz - ru * uz;
        if (sqrt(wx * wx + wy * wy + wz * wz) <= 1e-9 * L3) {
            // the discrete joint is on the line: a fixed perpendicular, u x (the axis
            // least aligned with u)
            const double ax = fabs(ux), ay = fabs(uy), az_ = fabs(uz);
            const int ix = (ax <= ay && ax <= az_) ? 0 : (ay <= az_ ? 1 : 2);
            const double ex = ix == 0, ey = ix == 1, ez = ix == 2;
            wx = uy * ez - uz * ey;
            wy = uz * ex - ux * ez;
            wz = ux * ey - uy * ex;
        }
        const double wn = sqrt(wx * wx + wy * wy + wz * wz);
        wx /= wn;
        wy /= wn;
        wz /= wn;
        const double Jx = px + aa * ux + h * wx, Jy = py + aa * uy + h * wy, Jz = pz + aa * uz + h * wz;
        double a3, e3, a4, e4;
        angles_near(Jx - px, Jy - py, Jz - pz, az3, el3, a3, e3);
        angles_near(tx - Jx, ty - Jy, tz - Jz, az4, el4, a4, e4);
        oi[n - 4] = a.type[n - 4] == 0 ? a3 - paz : e3 - pel;
        oi[n - 3] = a.type[n - 3] == 0 ? a3 - paz : e3 - pel;
        oi[n - 2] = a.type[n - 2] == 0 ? a4 - a3 : e4 - e3;
        oi[n - 1] = a.type[n - 1] == 0 ? a4 - a3 : e4 - e3;
        status[i] = 0;
    }
}

hipError_t launch_refine(const RefineArgs& a, const int32_t* q_steps, const double* targets, int64_t count,
                         double* angles, int32_t* status, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine, dim3(grid_for((uint64_t)count)), dim3(kBlock), 0, st, a, q_steps, targets, count,
                       angles, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reach poses (Step 3): depth-first walk from the root over the joint angles in the
// canonical order (distance to the reference angle, then value), stepping only into
// states that extend to a full solution (D_k on the forward side, B_k on the
// backward side).  Every such state has at least one valid child, so the walk emits
// the solutions in lexicographic order; it stops after `want` of them.  One block:
// the candidates of a node are tested in parallel, one lane per angle.
// ---------------------------------------------------------------------------
constexpr int kDfsThreads = 64;      // one wave: barriers cost next to nothing

__global__ void __launch_bounds__(kDfsThreads) k_dfs(DfsArgs a) {
    __shared__ short order[kMaxDof][kMaxNa + 1];
    __shared__ int olen[kMaxDof];
    __shared__ uint64_t state[kMaxDof + 1];
    __shared__ uint64_t cmask[kMaxDof][4];
    __shared__ uint64_t nextk[kMaxDof][kMaxNa];   // the state each accepted candidate leads to
    __shared__ int pick[kMaxDof];
    __shared__ int depth, nsol, done, need_eval;
    __shared__ long long steps;
    const int tid = threadIdx.x;
    const int na = a.na;
    for (int k = 0; k < a.n; ++k) {
        const JointView J = a.joints[k];
        const int L = J.hi - J.lo + 1;
        const int ref = a.ref[k];
        for (int t = tid; t < L; t += blockDim.x) {
            int v = J.lo + t;
            int dv = abs(v - ref);
            int rank = 0;
            for (int u = J.lo; u <= J.hi; ++u) {
                int du = abs(u - ref);
                if (du < dv || (du == dv && u < v)) ++rank;
            }
            order[k][rank] = (short)v;
        }
        if (tid == 0) olen[k] = L;
    }
    if (tid == 0) {
        state[0] = a.root;
        depth = 0;
        nsol = 0;
        done = 0;
        need_eval = 1;
        steps = 0;
    }
    __syncthreads();
    while (true) {
        if (need_eval) {
            // one wave; lane l takes candidates l, l + 64, ...  The membership probe and
            // the segment test are both issued (no short cut), so that their loads overlap.
            const int d = depth;
            const JointView J = a.joints[d];
            int x, y, z, ia, ie;
            unpack_key(state[d], x, y, z, ia, ie);
            for (int c0 = 0; c0 < olen[d]; c0 += kDfsThreads) {
                const int c = c0 + tid;
                bool ok = false;
                if (c < olen[d]) {
                    const int av = order[d][c];
                    int ia2 = ia, ie2 = ie;
                    if (J.type == 0)
                        ia2 = wrap_na(ia + av, na);
                    else
                        ie2 = wrap_na(ie + av, na);
                    const int o = ia2 * na + ie2;
                    const short4 dd = J.off[o];
                    const uint64_t key = pack_key(x + dd.x, y + dd.y, z + dd.z, ia2, ie2);
                    const bool mem = set_member(a.sets[d + 1], key);
                    const bool clear = segment_clear_all(a.g, J, o, x, y, z);
                    ok = mem && clear;
                    if (ok) nextk[d][c] = key;
                }
                const unsigned long long b = __ballot(ok);
                if (tid == 0) cmask[d][c0 >> 6] = b;
            }
            if (tid == 0)
                for (int w = (olen[d] + 63) >> 6; w < 4; ++w) cmask[d][w] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            need_eval = 0;
            while (true) {
                // every state offered to the walk extends to a solution, so a walk
                // needs at most n steps per solution; a much longer one is an error
                if (++steps > (long long)(a.want + 1) * 4096 * (a.n + 1)) {
                    nsol = -1;
                    done = 1;
                    break;
                }
                if (depth == a.n) {
                    for (int k = 0; k < a.n; ++k) a.sols[nsol * a.n + k] = pick[k];
                    ++nsol;
                    if (nsol >= a.want) {
                        done = 1;
                        break;
                    }
                    --depth;
                    continue;
                }
                int j = -1;
                for (int w = 0; w < 4; ++w) {
                    if (cmask[depth][w]) {
                        int b = __ffsll((unsigned long long)cmask[depth][w]) - 1;
                        cmask[depth][w] &= cmask[depth][w] - 1;
                        j = 64 * w + b;
                        break;
                    }
                }
                if (j < 0) {
                    if (depth == 0) {
                        done = 1;
                        break;
                    }
                    --depth;
                    continue;
                }
                pick[depth] = order[depth][j];
                state[depth + 1] = nextk[depth][j];
                ++depth;
                if (depth < a.n) {
                    need_eval = 1;
                    break;
                }
            }
            *a.nsol = nsol;
        }
        __syncthreads();
        if (done) break;
    }
}

hipError_t launch_dfs(const DfsArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_dfs, dim3(1), dim3(kDfsThreads), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pose replay: one thread per pose.
// ---------------------------------------------------------------------------
template <class Args>
__device__ bool replay(const Args& a, const int32_t* q, int32_t* end) {
    int x = a.bx, y = a.by, z = a.bz, ia = a.ia0, ie = a.ie0;
    bool ok = cell_free(a.g, x, y, z);
    for (int k = 0; k < a.n; ++k) {
        const JointView J = a.joints[k];
        if (J.type == 0)
            ia = wrap_na(ia + q[k], a.na);
        else
            ie = wrap_na(ie + q[k], a.na);
        int o = ia * a.na + ie;
        if (ok && !segment_clear(a.g, J, o, x, y, z)) ok = false;
        short4 d = J.off[o];
        x += d.x;
        y += d.y;
        z += d.z;
    }
    if (end) {
        end[0] = x;
        end[1] = y;
        end[2] = z;
    }
    return ok;
}

__global__ void k_pose_check(PoseArgs a, const int32_t* q, int64_t count, uint8_t* valid, int32_t* ends) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool ok = replay(a, q + i * a.n, ends ? ends + i * 3 : nullptr);
        valid[i] = ok ? 1 : 0;
    }
}

// The same for a few poses, one wave per pose: lane k takes segment k.  Its orientation
// is the sum of the joint steps before it, its start the prefix sum of the earlier end
// offsets (a scan over the lanes), so the segments are tested together instead of one
// after another.
__global__ void __launch_bounds__(64) k_pose_check_wave(PoseArgs a, const int32_t* q, int64_t count,
                                                        uint8_t* valid, int32_t* ends) {
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= count) return;
    const int32_t* qi = q + i * a.n;
    const bool live = lane < a.n;
    int o = 0, dx = 0, dy = 0, dz = 0;
    if (live) {
        int ia = a.ia0, ie = a.ie0;
        for (int k = 0; k <= lane; ++k) {
            if (a.joints[k].type == 0)
                ia = wrap_na(ia + qi[k], a.na);
            else
                ie = wrap_na(ie + qi[k], a.na);
        }
        o = ia * a.na + ie;
        const short4 d = a.joints[lane].off[o];
        dx = d.x;
        dy = d.y;
        dz = d.z;
    }
    // inclusive scan of the offsets over the lanes; the segment starts at the exclusive sum
    int sx = dx, sy = dy, sz = dz;
    for (int off = 1; off < 64; off <<= 1) {
        const int tx = __shfl_up(sx, off, 64), ty = __shfl_up(sy, off, 64), tz = __shfl_up(sz, off, 64);
        if (lane >= off) {
            sx += tx;
            sy += ty;
            sz += tz;
        }
    }
    const int x = a.bx + sx - dx, y = a.by + sy - dy, z = a.bz + sz - dz;
    bool ok = true;
    if (live) ok = segment_clear_all(a.g, a.joints[lane], o, x, y, z);
    if (lane == 0) ok = ok && cell_free(a.g, a.bx, a.by, a.bz);
    const bool all = __ballot(!ok) == 0;
    if (lane == a.n - 1) {
        valid[i] = all ? 1 : 0;
        if (ends) {
            ends[i * 3] = a.bx + sx;
            ends[i * 3 + 1] = a.by + sy;
            ends[i * 3 + 2] = a.bz + sz;
        }
    }
}

hipError_t launch_pose_check(const PoseArgs& a, const int32_t* q, int64_t count, uint8_t* valid, int32_t* ends,
                             hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (count <= 64 && a.n >= 1)
        hipLaunchKernelGGL(k_pose_check_wave, dim3((uint32_t)count), dim3(64), 0, st, a, q, count, valid, ends);
    else
        hipLaunchKernelGGL(k_pose_check, dim3(grid_for((uint64_t)count)), dim3(kBlock), 0, st, a, q, count, valid,
                           ends);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The paper's gap search ("The gap in gMS", "The procedure for IK solution"): arm
// positions stay numerical (FP64); a segment is tested at its S sample points rounded to
// voxels.  Every decision is made with the same multiplies and adds, in the same order,
// as the host-side definition: no contraction into fused multiply-adds, no square root.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long gms_round(double v) {
#pragma clang fp contract(off)
    const double a = fabs(v);
    const double f = floor(a);
    const double frac = a - f;
    const double r = (frac > 0.5 || fabs(frac - 0.5) <= 1e-9) ? f + 1.0 : f;
    return v >= 0 ? (long long)r : -(long long)r;
}

// Segment from p along w: samples p + t_s w clear (in the grid and free).
__device__ bool gms_clear(const GmsArgs& a, double px, double py, double pz, double wx, double wy, double wz) {
#pragma clang fp contract(off)
    for (int s = 0; s < a.S; ++s) {
        const double t = a.ts[s];
        const long long x = gms_round(px + t * wx), y = gms_round(py + t * wy), z = gms_round(pz + t * wz);
        if (x < 0 || y < 0 || z < 0 || x >= a.g.n || y >= a.g.n || z >= a.g.n) return false;
        if (!cell_free(a.g, (int)x, (int)y, (int)z)) return false;
    }
    return true;
}

__device__ __forceinline__ bool gms_flex(double dot, double c, double n2) {
#pragma clang fp contract(off)
    if (c >= 0) return dot >= 0 && dot * dot >= (c * c) * n2;
    return dot >= 0 || dot * dot <= (c * c) * n2;
}

__global__ void __launch_bounds__(kBlock) k_gms_flags(GmsArgs a, uint8_t* flags1, uint8_t* flags4) {
#pragma clang fp contract(off)
    // the base and the target voxel must be free
    const bool ends = cell_free(a.g, (int)a.p0[0], (int)a.p0[1], (int)a.p0[2]) &&
                      cell_free(a.g, (int)a.t[0], (int)a.t[1], (int)a.t[2]);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < a.nq; q += gridDim.x * blockDim.x) {
        const double rx = a.Q[3 * q], ry = a.Q[3 * q + 1], rz = a.Q[3 * q + 2];
        // Step 1: joint-1 limit, eq 5, collision
        bool ok1 = ends && rz >= a.min_el;
        if (ok1) {
            const double x1 = a.p0[0] + a.L1 * rx, y1 = a.p0[1] + a.L1 * ry, z1 = a.p0[2] + a.L1 * rz;
            const double dx = x1 - a.t[0], dy = y1 - a.t[1], dz = z1 - a.t[2];
            ok1 = dx * dx + dy * dy + dz * dz <= a.r5sq;
            ok1 = ok1 && gms_clear(a, a.p0[0], a.p0[1], a.p0[2], a.L1 * rx, a.L1 * ry, a.L1 * rz);
        }
        flags1[q] = ok1 ? 1 : 0;
        // segment 4 backward from the target: inside the cone, clear
        bool ok4 = ends && (!a.has_cone || rx * a.ax[0] + ry * a.ax[1] + rz * a.ax[2] >= a.cone_c);
        if (ok4) {
            const double wx = a.L4 * rx, wy = a.L4 * ry, wz = a.L4 * rz;
            ok4 = gms_clear(a, a.t[0] - wx, a.t[1] - wy, a.t[2] - wz, wx, wy, wz);
        }
        flags4[q] = ok4 ? 1 : 0;
    }
}

hipError_t launch_gms_flags(const GmsArgs& a, uint8_t* flags1, uint8_t* flags4, hipStream_t st) {
    hipLaunchKernelGGL(k_gms_flags, dim3(grid_for((uint64_t)a.nq)), dim3(kBlock), 0, st, a, flags1, flags4);
    return hipGetLastError();
}

// The segment-4 list in cluster order: pts[k] = (t - L4 r_l, l) for l = order[k].
__global__ void k_gms_points(GmsArgs a, const int32_t* __restrict__ order, int n4, GmsPoint* pts) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n4) return;
    const int l = order[k];
    GmsPoint p;
    p.x = a.t[0] - a.L4 * a.Q[3 * l];
    p.y = a.t[1] - a.L4 * a.Q[3 * l + 1];
    p.z = a.t[2] - a.L4 * a.Q[3 * l + 2];
    p.l = l;
    p.pad = 0;
    pts[k] = p;
}

hipError_t launch_gms_points(const GmsArgs& a, const int32_t* order, int n4, GmsPoint* pts, hipStream_t st) {
    if (n4 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gms_points, dim3((n4 + 255) / 256), dim3(256), 0, st, a, order, n4, pts);
    return hipGetLastError();
}

// Candidates of one wave that passed the free vector's length and flexion tests, waiting
// for segment 3's sample test: at most 63 wait between drains and 64 arrive per pass.
struct GmsQueue {
    double px[128], py[128], pz[128], vx[128], vy[128], vz[128];
    uint64_t key[128];
    int32_t ii[128];
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Segment 3's samples for queue entries [start, start + n), one per lane; the solutions
// are counted per survivor and, while there is room, their keys stored.
__device__ void gms_drain(const GmsArgs& a, GmsQueue& q, int start, int n, int lane, unsigned long long* slots,
                          unsigned long long* per_i, uint64_t* keys, uint64_t cap, bool& room) {
    wave_sync();
    bool sol = false;
    int ii = -1;
    uint64_t key = 0;
    if (lane < n) {
        const int e = start + lane;
        ii = q.ii[e];
        key = q.key[e];
        sol = gms_clear(a, q.px[e], q.py[e], q.pz[e], q.vx[e], q.vy[e], q.vz[e]);
    }
    wave_sync();
    const unsigned long long got = __ballot(sol);
    for (unsigned long long todo = got; todo;) {
        const int x = __shfl(ii, __ffsll((long long)todo) - 1, 64);
        const unsigned long long same = __ballot(sol && ii == x);
        if (lane == 0) atomicAdd(&per_i[x], (unsigned long long)__popcll(same));
        todo &= ~same;
    }
    if (room && got) {
        unsigned long long first = 0;
        if (lane == 0) first = atomicAdd(slots, (unsigned long long)__popcll(got));
        first = __shfl(first, 0, 64);
        if (first >= cap) room = false;
        const uint64_t slot = first + (uint64_t)__popcll(got & ((1ull << lane) - 1));
        if (sol && slot < cap) keys[slot] = key;
    }
}

// Steps 2A/2B.  Each lane of a wave first tests one (survivor ii, quiver vector j) pair:
// joint-2 limit, p2, eq 7, segment 2's samples.  The wave then takes its surviving pairs
// one at a time, all 64 lanes over the segment-4 list: a lane tests one cluster of
// kGmsCluster points against the pair's p2 (the cluster's bounds on |p3 - p2|, widened,
// against the gap's length: a skipped cluster holds no point that passes the exact test),
// then four kept clusters are taken per pass, one point per lane, with the exact tests of
// the free vector's length and the joint 3 and 4 limits (on squares).  Candidates that
// pass wait in the wave's queue in LDS; 64 at a time take segment 3's sample test, so
// that the longest test runs on full waves.  Solutions are counted per survivor from the
// wave's ballots; the wave reserves key slots with one atomic per ballot until the key
// array is full.
__global__ void __launch_bounds__(kBlock) k_gms_pairs(GmsArgs a, const int32_t* __restrict__ s1, int n1,
                                                      const GmsPoint* __restrict__ pts, int n4,
                                                      const GmsCluster* __restrict__ cl, int ncl,
                                                      unsigned long long* slots, unsigned long long* per_i,
                                                      uint64_t* keys, uint64_t cap, int min_ii, int max_ii,
                                                      int store) {
#pragma clang fp contract(off)
    __shared__ GmsQueue queues[kBlock / 64];
    const int lane = threadIdx.x & 63;
    GmsQueue& q = queues[threadIdx.x >> 6];
    int qn = 0;
    const uint64_t total = (uint64_t)(min(n1, max_ii + 1) - min_ii) * (uint64_t)a.nq;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool room = store != 0;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x - lane); base < total; base += stride) {
        const uint64_t idx = base + lane;
        bool live = idx < total;
        int ii = 0, j = 0;
        double x2 = 0, y2 = 0, z2 = 0, rjx = 0, rjy = 0, rjz = 0;
        if (live) {
            const int di = (int)(idx / (uint64_t)a.nq);
            j = (int)(idx - (uint64_t)di * a.nq);
            ii = min_ii + di;
            const int i = s1[ii];
            const double rix = a.Q[3 * i], riy = a.Q[3 * i + 1], riz = a.Q[3 * i + 2];
            rjx = a.Q[3 * j];
            rjy = a.Q[3 * j + 1];
            rjz = a.Q[3 * j + 2];
            live = rix * rjx + riy * rjy + riz * rjz >= a.c1;    // joint 2 limit
            if (live) {
                const double x1 = a.p0[0] + a.L1 * rix, y1 = a.p0[1] + a.L1 * riy, z1 = a.p0[2] + a.L1 * riz;
                x2 = x1 + a.L2 * rjx;
                y2 = y1 + a.L2 * rjy;
                z2 = z1 + a.L2 * rjz;
                const double dx = x2 - a.t[0], dy = y2 - a.t[1], dz = z2 - a.t[2];
                live = dx * dx + dy * dy + dz * dz <= a.r7sq;       // eq 7
                live = live && gms_clear(a, x1, y1, z1, a.L2 * rjx, a.L2 * rjy, a.L2 * rjz);
            }
        }
        unsigned long long pending = __ballot(live);
        while (pending) {
            const int src = __ffsll((long long)pending) - 1;
            pending &= pending - 1;
            const double px = __shfl(x2, src, 64), py = __shfl(y2, src, 64), pz = __shfl(z2, src, 64);
            const double ux = __shfl(rjx, src, 64), uy = __shfl(rjy, src, 64), uz = __shfl(rjz, src, 64);
            const int pii = __shfl(ii, src, 64), pj = __shfl(j, src, 64);
            const uint64_t pkey = ((uint64_t)s1[pii] << 40) | ((uint64_t)pj << 20);
            for (int c0 = 0; c0 < ncl; c0 += 64) {
                bool keep = false;
                if (c0 + lane < ncl) {
                    const GmsCluster& C = cl[c0 + lane];
                    const double dx = C.cx - px, dy = C.cy - py, dz = C.cz - pz;
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    keep = d2 >= C.lo2 && d2 <= C.hi2;
                }
                unsigned long long kept = __ballot(keep);
                while (kept) {
                    // up to four kept clusters, one per quarter of the wave
                    int pick = -1;
                    for (int r = 0; r < 4 && kept; ++r) {
                        const int b = __ffsll((long long)kept) - 1;
                        kept &= kept - 1;
                        if ((lane >> 4) == r) pick = b;
                    }
                    bool cand = false;
                    double vx = 0, vy = 0, vz = 0;
                    int l = 0;
                    const int k = (c0 + pick) * kGmsCluster + (lane & (kGmsCluster - 1));
                    if (pick >= 0 && k < n4) {
                        const GmsPoint P = pts[k];
                        vx = P.x - px;
                        vy = P.y - py;
                        vz = P.z - pz;
                        const double n2 = vx * vx + vy * vy + vz * vz;
                        if (n2 >= a.glo && n2 <= a.ghi) {                    // the gap's free vector
                            l = P.l;
                            const double rlx = a.Q[3 * l], rly = a.Q[3 * l + 1], rlz = a.Q[3 * l + 2];
                            cand = gms_flex(ux * vx + uy * vy + uz * vz, a.c2, n2) &&     // joint 3 limit
                                   gms_flex(vx * rlx + vy * rly + vz * rlz, a.c3, n2);    // joint 4 limit
                        }
                    }
                    const unsigned long long cm = __ballot(cand);
                    if (cm) {
                        if (cand) {
                            const int e = qn + __popcll(cm & ((1ull << lane) - 1));
                            q.px[e] = px;
                            q.py[e] = py;
                            q.pz[e] = pz;
                            q.vx[e] = vx;
                            q.vy[e] = vy;
                            q.vz[e] = vz;
                            q.key[e] = pkey | (uint64_t)l;
                            q.ii[e] = pii;
                        }
                        qn += __popcll(cm);
                        if (qn >= 64) {
                            qn -= 64;
                            gms_drain(a, q, qn, 64, lane, slots, per_i, keys, cap, room);
                        }
                    }
                }
            }
        }
    }
    if (qn > 0) gms_drain(a, q, 0, qn, lane, slots, per_i, keys, cap, room);
}

hipError_t launch_gms_pairs(const GmsArgs& a, const int32_t* s1, int n1, const GmsPoint* pts, int n4,
                            const GmsCluster* cl, int ncl, unsigned long long* slots, unsigned long long* per_i,
                            uint64_t* keys, uint64_t cap, int min_ii, int max_ii, int store, hipStream_t st) {
    const int hi = std::min(n1, max_ii + 1);
    if (min_ii < 0 || hi <= min_ii || n4 == 0) return hipSuccess;
    const uint64_t work = (uint64_t)(hi - min_ii) * (uint64_t)a.nq;
    hipLaunchKernelGGL(k_gms_pairs, dim3(grid_for(work, kBlock, 65536)), dim3(kBlock), 0, st, a, s1, n1, pts, n4, cl,
                       ncl, slots, per_i, keys, cap, min_ii, max_ii, store);
    return hipGetLastError();
}

// s1, s2, v3, s4 of a solution and the exact s3 = v3 L3 / |v3|, s4' = (t - p2) - s3.
__global__ void k_gms_vectors(GmsArgs a, const uint64_t* keys, int n, double* out) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint64_t key = keys[k];
    const int i = (int)(key >> 40), j = (int)((key >> 20) & 0xfffff), l = (int)(key & 0xfffff);
    const double* ri = a.Q + 3 * i;
    const double* rj = a.Q + 3 * j;
    const double* rl = a.Q + 3 * l;
    double* o = out + (size_t)k * 18;
    double p2[3], v3[3];
    for (int c = 0; c < 3; ++c) {
        const double p1 = a.p0[c] + a.L1 * ri[c];
        p2[c] = p1 + a.L2 * rj[c];
        v3[c] = (a.t[c] - a.L4 * rl[c]) - p2[c];
        o[c] = a.L1 * ri[c];
        o[3 + c] = a.L2 * rj[c];
        o[6 + c] = v3[c];
        o[9 + c] = a.L4 * rl[c];
    }
    const double n3 = sqrt(v3[0] * v3[0] + v3[1] * v3[1] + v3[2] * v3[2]);
    for (int c = 0; c < 3; ++c) {
        const double s3 = v3[c] * a.L3 / n3;
        o[12 + c] = s3;
        o[15 + c] = (a.t[c] - p2[c]) - s3;
    }
}

hipError_t launch_gms_vectors(const GmsArgs& a, const uint64_t* keys, int n, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gms_vectors, dim3((n + 63) / 64), dim3(64), 0, st, a, keys, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Short-reach shortcut ("Short Reaches"): a segment hypothesis (a state of F_{k-1} and an
// angle of joint k) hits the target at its first sample within rho of the target when
// every earlier sample is free and in the grid; the shortest hit wins.
// ---------------------------------------------------------------------------
// Hit key of one hypothesis from (x, y, z) along orientation o, or ~0 for no hit; *hs
// receives the hit sample (1-based).
__device__ __forceinline__ unsigned long long hit_key(const HitArgs& h, const JointView& j, int o, int x, int y,
                                                      int z, int* hs = nullptr) {
    const short4* sw = j.sweep + (size_t)o * j.S;
    for (int s = 0; s < j.S; ++s) {
        const short4 d = sw[s];
        const int px = x + d.x, py = y + d.y, pz = z + d.z;
        if (!cell_free(h.g, px, py, pz)) return ~0ull;
        const int ex = px - h.tx, ey = py - h.ty, ez = pz - h.tz;
        const int d2 = ex * ex + ey * ey + ez * ez;
        if (d2 <= h.rho2) {
            if (hs) *hs = s + 1;
            const unsigned long long len = (unsigned long long)(h.base_len + (long long)(s + 1) * h.len);
            return (len << 40) | ((unsigned long long)d2 << 24) | ((unsigned long long)h.k << 16);
        }
    }
    return ~0ull;
}

// Orientation after joint j turns (ia, ie) by a.
__device__ __forceinline__ int turn_o(const JointView& j, int na, int ia, int ie, int a) {
    if (j.type == 0)
        ia = wrap_na(ia + a, na);
    else
        ie = wrap_na(ie + a, na);
    return ia * na + ie;
}

__global__ void __launch_bounds__(kBlock) k_hits(const uint64_t* __restrict__ in, uint64_t count, JointView j,
                                                 HitArgs h, unsigned long long* best) {
    const uint32_t nA = (uint32_t)(j.hi - j.lo + 1);
    unsigned long long mine = ~0ull;
    const uint64_t total = count * (uint64_t)nA;
    for (uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = idx / nA;
        const int a = j.lo + (int)(idx - i * nA);
        int x, y, z, ia, ie;
        unpack_key(in[i], x, y, z, ia, ie);
        if (ia >= h.na || ie >= h.na) continue;
        const unsigned long long key = hit_key(h, j, turn_o(j, h.na, ia, ie, a), x, y, z);
        mine = key < mine ? key : mine;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(mine, off, 64);
        mine = o < mine ? o : mine;
    }
    if ((threadIdx.x & 63) == 0 && mine != ~0ull) atomicMin(best, mine);
}

hipError_t launch_hits(const uint64_t* in, uint64_t count, JointView j, HitArgs h, unsigned long long* best,
                       hipStream_t st) {
    const uint64_t work = count * (uint64_t)(j.hi - j.lo + 1);
    if (work == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hits, dim3(grid_for(work)), dim3(kBlock), 0, st, in, count, j, h, best);
    return hipGetLastError();
}

// One thread per state of the list: kept when some angle gives the best key.
__global__ void __launch_bounds__(kBlock) k_hit_mark(const uint64_t* __restrict__ in, uint64_t count, SetView fprev,
                                                     JointView j, HitArgs h, const unsigned long long* best) {
    const unsigned long long want = *best;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = in[i];
        int x, y, z, ia, ie;
        unpack_key(key, x, y, z, ia, ie);
        bool keep = false;
        if (ia < h.na && ie < h.na)
            for (int a = j.lo; a <= j.hi && !keep; ++a)
                keep = hit_key(h, j, turn_o(j, h.na, ia, ie, a), x, y, z) == want;
        if (!keep) set_remove(fprev, key);
    }
}

hipError_t launch_hit_mark(const uint64_t* in, uint64_t count, SetView fprev, JointView j, HitArgs h,
                           const unsigned long long* best, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hit_mark, dim3(grid_for(count)), dim3(kBlock), 0, st, in, count, fprev, j, h, best);
    return hipGetLastError();
}

// One wave: at joint j (0-based) the lanes try the window's angles 64 at a time in the
// canonical order (|a| then a); the first that steps into D_{j+1} with a clear segment
// (or, at the hit's joint, gives the best key) is taken.
__global__ void __launch_bounds__(64) k_hit_walk(HitWalkArgs a) {
    __shared__ int order[kMaxNa];
    const int lane = threadIdx.x;
    const unsigned long long want = *a.best;
    const int k = (int)((want >> 16) & 0xff);
    int x = a.bx, y = a.by, z = a.bz, ia = a.ia0, ie = a.ie0;
    for (int jj = 0; jj < k; ++jj) {
        const JointView& J = a.joints[jj];
        if (lane == 0) {
            // the window in the canonical order: 0, -1, +1, -2, +2, ... inside [lo, hi]
            const int nw = J.hi - J.lo + 1;
            int m = 0;
            if (J.lo <= 0 && 0 <= J.hi) order[m++] = 0;
            for (int d = 1; m < nw; ++d) {
                if (-d >= J.lo && -d <= J.hi) order[m++] = -d;
                if (d >= J.lo && d <= J.hi) order[m++] = d;
            }
        }
        __syncthreads();
        const int nA = J.hi - J.lo + 1;
        int pick = -1, pick_s = 0;
        for (int base = 0; base < nA && pick < 0; base += 64) {
            const int r = base + lane;
            bool ok = false;
            int s_hit = 0;
            if (r < nA) {
                const int ang = order[r];
                const int o = turn_o(J, a.na, ia, ie, ang);
                if (jj == k - 1) {
                    ok = hit_key(a.h, J, o, x, y, z, &s_hit) == want;
                } else {
                    const short4 d = J.off[o];
                    const int o_ia = o / a.na, o_ie = o % a.na;
                    ok = set_member(a.D[jj + 1], pack_key(x + d.x, y + d.y, z + d.z, o_ia, o_ie)) &&
                         segment_clear_all(a.h.g, J, o, x, y, z);
                }
            }
            const uint64_t bal = __ballot(ok);
            if (bal) {
                const int first = __ffsll((long long)bal) - 1;
                pick = base + first;
                pick_s = __shfl(s_hit, first, 64);
            }
        }
        if (pick < 0) {
            if (lane == 0) a.out[kMaxDof] = -1;
            return;
        }
        const int ang = order[pick];
        const int o = turn_o(J, a.na, ia, ie, ang);
        if (lane == 0) a.out[jj] = ang;
        if (jj == k - 1) {
            if (lane == 0) a.out[kMaxDof] = pick_s;
            return;
        }
        const short4 d = J.off[o];
        x += d.x;
        y += d.y;
        z += d.z;
        ia = o / a.na;
        ie = o % a.na;
        __syncthreads();   // order is rewritten for the next joint
    }
}

hipError_t launch_hit_walk(const HitWalkArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_hit_walk, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Waypoint tracking ("Smooth sequence computation", "Filtering for smoothness", "Path
// between Arbitrary Poses").  One block per query, persistent over the waypoints of
// every candidate solution.  At a waypoint the block scores the joint box of radius d
// around the current pose: candidate c enumerates the box in the canonical order (digit
// k of c in base 2d + 1, joint 1 most significant, digit r <-> change t in the order
// 0, -1, +1, -2, +2, ...), so the order key is (L1 change, squared distance, c) and the
// pose is the block's minimum key among the poses that are valid and within the
// tolerance.  The tracked joint's distance is tested first; only candidates within the
// tolerance replay the whole arm against the grid.
// ---------------------------------------------------------------------------
constexpr int kTrackThreads = 512;

__device__ __forceinline__ int track_change(int r) { return r == 0 ? 0 : ((r & 1) ? -((r + 1) >> 1) : (r >> 1)); }

// Minimum key over the box of radius d around q (all threads return it).  The box is
// split at the tracked joint: a thread takes prefixes (the changes of joints
// 1..tracked, the high digits of c), tests the tracked joint's distance and the prefix
// segments once, and only then walks the suffixes (the remaining joints) of a prefix
// that passed.
__device__ unsigned long long track_best(const TrackArgs& a, const int* q, int d, int px, int py, int pz,
                                         bool base_free, unsigned long long* red) {
    const int n = a.n, tr = a.tracked;
    const uint64_t B = (uint64_t)(2 * d + 1);
    uint64_t total_p = 1, total_s = 1;
    for (int k = 0; k < tr; ++k) total_p *= B;
    for (int k = tr; k < n; ++k) total_s *= B;
    unsigned long long best = ~0ull;
    for (uint64_t pi = threadIdx.x; pi < total_p && base_free; pi += blockDim.x) {
        int tp[kMaxDof];
        uint64_t rest = pi;
        bool inside = true;
        int l1p = 0;
        for (int k = tr - 1; k >= 0; --k) {
            tp[k] = track_change((int)(rest % B));
            rest /= B;
            const int v = q[k] + tp[k];
            inside = inside && v >= a.lim_lo[k] && v <= a.lim_hi[k];
            l1p += tp[k] < 0 ? -tp[k] : tp[k];
        }
        if (!inside) continue;
        // the tracked joint: offsets only
        int ia = a.ia0, ie = a.ie0, x = a.bx, y = a.by, z = a.bz;
        for (int k = 0; k < tr; ++k) {
            if (a.joints[k].type == 0)
                ia = wrap_na(ia + q[k] + tp[k], a.na);
            else
                ie = wrap_na(ie + q[k] + tp[k], a.na);
            const short4 o = a.joints[k].off[ia * a.na + ie];
            x += o.x;
            y += o.y;
            z += o.z;
        }
        const int dx = x - px, dy = y - py, dz = z - pz;
        const int d2 = dx * dx + dy * dy + dz * dz;
        if (d2 > a.eps2) continue;
        const unsigned long long head = ((unsigned long long)d2 << 42) | (unsigned long long)(pi * total_s);
        if (((unsigned long long)l1p << 52 | head) >= best) continue;   // no suffix can do better
        // the prefix segments against the grid
        ia = a.ia0;
        ie = a.ie0;
        x = a.bx;
        y = a.by;
        z = a.bz;
        bool clear = true;
        for (int k = 0; k < tr && clear; ++k) {
            const JointView& J = a.joints[k];
            if (J.type == 0)
                ia = wrap_na(ia + q[k] + tp[k], a.na);
            else
                ie = wrap_na(ie + q[k] + tp[k], a.na);
            const int o = ia * a.na + ie;
            clear = segment_clear_all(a.g, J, o, x, y, z);
            const short4 off = J.off[o];
            x += off.x;
            y += off.y;
            z += off.z;
        }
        if (!clear) continue;
        // the suffixes, in canonical order
        for (uint64_t si = 0; si < total_s; ++si) {
            int ts[kMaxDof];
            uint64_t r2 = si;
            bool in2 = true;
            int l1 = l1p;
            for (int k = n - 1; k >= tr; --k) {
                ts[k] = track_change((int)(r2 % B));
                r2 /= B;
                const int v = q[k] + ts[k];
                in2 = in2 && v >= a.lim_lo[k] && v <= a.lim_hi[k];
                l1 += ts[k] < 0 ? -ts[k] : ts[k];
            }
            if (!in2) continue;
            const unsigned long long key = ((unsigned long long)l1 << 52) | (head + si);
            if (key >= best) continue;
            int sia = ia, sie = ie, sx = x, sy = y, sz = z;
            bool ok = true;
            for (int k = tr; k < n && ok; ++k) {
                const JointView& J = a.joints[k];
                if (J.type == 0)
                    sia = wrap_na(sia + q[k] + ts[k], a.na);
                else
                    sie = wrap_na(sie + q[k] + ts[k], a.na);
                const int o = sia * a.na + sie;
                ok = segment_clear_all(a.g, J, o, sx, sy, sz);
                const short4 off = J.off[o];
                sx += off.x;
                sy += off.y;
                sz += off.z;
            }
            if (ok) best = key;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    __syncthreads();   // red may still be read by the previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    best = ~0ull;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) best = red[w] < best ? red[w] : best;
    return best;
}

__device__ void track_body(const TrackArgs& a) {
    __shared__ int pts[kTrackMaxPoints * 3];
    __shared__ int qc[kMaxDof];
    __shared__ int seg[kMaxDof * 4];   // orientation and start voxel of each segment
    __shared__ unsigned long long red[kTrackThreads / 64];
    __shared__ int npts;
    const int n = a.n;
    const bool base_free = cell_free(a.g, a.bx, a.by, a.bz);
    if (threadIdx.x == 0) {
        a.status[0] = 0;
        a.status[1] = -1;
        a.status[2] = 0;
    }
    for (int i = 0; i < a.nsol; ++i) {
        const int width = a.mode == 1 ? a.vn : n;
        const int32_t* sol = a.sols + (size_t)i * width;
        if (threadIdx.x == 0) {
            // the pose whose sample points are the waypoints: the reach pose (mode 0), the
            // virtual arm's pose (mode 1) or the shortcut's joint prefix (mode 2)
            const bool virt = a.mode == 1;
            const JointView* J = virt ? a.vjoints : a.joints;
            const int* len = virt ? a.vlen : a.len;
            const int* src = a.mode == 2 ? a.guide : sol;
            const int sn = a.mode == 2 ? a.guide_k : width;
            int ia = virt ? a.via0 : a.ia0, ie = virt ? a.vie0 : a.ie0;
            int x = virt ? a.vbx : a.bx, y = virt ? a.vby : a.by, z = virt ? a.vbz : a.bz;
            for (int k = 0; k < sn; ++k) {
                if (J[k].type == 0)
                    ia = wrap_na(ia + src[k], a.na);
                else
                    ie = wrap_na(ie + src[k], a.na);
                const int o = ia * a.na + ie;
                seg[4 * k] = o;
                seg[4 * k + 1] = x;
                seg[4 * k + 2] = y;
                seg[4 * k + 3] = z;
                const short4 off = J[k].off[o];
                x += off.x;
                y += off.y;
                z += off.z;
            }
            int m = 0;
            auto push = [&](int k, int s) {
                const short4 d = J[k].sweep[(size_t)seg[4 * k] * J[k].S + s];
                pts[3 * m] = seg[4 * k + 1] + d.x;
                pts[3 * m + 1] = seg[4 * k + 2] + d.y;
                pts[3 * m + 2] = seg[4 * k + 3] + d.z;
                ++m;
            };
            if (a.mode == 0) {
                // segments tracked .. 2 from their ends back to their starts, then the end
                // of segment 1; the first point (the tracked joint itself) is left out
                bool first = true;
                for (int k = a.tracked - 1; k >= 1; --k) {
                    if (len[k] == 0) continue;
                    for (int s = J[k].S - 1; s >= 0; --s) {
                        if (first) {
                            first = false;
                            continue;
                        }
                        push(k, s);
                    }
                }
                if (!first) {
                    pts[3 * m] = seg[4 * 1 + 1];
                    pts[3 * m + 1] = seg[4 * 1 + 2];
                    pts[3 * m + 2] = seg[4 * 1 + 3];
                    ++m;
                }
            } else if (a.mode == 1) {
                for (int k = 0; k < sn; ++k) {
                    if (len[k] == 0) continue;
                    for (int s = 0; s < J[k].S; ++s) push(k, s);
                }
            } else {
                // the shortcut back from the target: the hit sample and the earlier ones of
                // segment k, segments k-1 .. 2 end to start, then the end of segment 1
                const int kk = a.guide_k - 1;
                for (int s = a.guide_s - 1; s >= 0; --s) push(kk, s);
                for (int k = kk - 1; k >= 1; --k) {
                    if (len[k] == 0) continue;
                    for (int s = J[k].S - 1; s >= 0; --s) push(k, s);
                }
                pts[3 * m] = seg[4 * 1 + 1];
                pts[3 * m + 1] = seg[4 * 1 + 2];
                pts[3 * m + 2] = seg[4 * 1 + 3];
                ++m;
            }
            npts = m;
        }
        const bool backward = a.mode != 1;
        if (threadIdx.x < n) qc[threadIdx.x] = backward ? sol[threadIdx.x] : a.start[threadIdx.x];
        __syncthreads();
        const int M = npts;
        if (threadIdx.x < n) a.rows[(size_t)(backward ? M : 0) * n + threadIdx.x] = qc[threadIdx.x];
        int w = 0;
        for (; w < M; ++w) {
            const int px = pts[3 * w], py = pts[3 * w + 1], pz = pts[3 * w + 2];
            int d = a.delta;
            unsigned long long best = track_best(a, qc, d, px, py, pz, base_free, red);
            if (best == ~0ull && a.delta2 != a.delta) {
                d = a.delta2;
                best = track_best(a, qc, d, px, py, pz, base_free, red);
            }
            if (best == ~0ull) break;
            __syncthreads();   // every thread has read qc
            if (threadIdx.x == 0) {
                uint64_t rest = best & ((1ull << 42) - 1);
                const uint64_t B = (uint64_t)(2 * d + 1);
                for (int k = n - 1; k >= 0; --k) {
                    qc[k] += track_change((int)(rest % B));
                    rest /= B;
                }
            }
            __syncthreads();
            const int row = backward ? M - 1 - w : w + 1;
            if (threadIdx.x < n) a.rows[(size_t)row * n + threadIdx.x] = qc[threadIdx.x];
        }
        if (threadIdx.x == 0) a.status[2] = w;
        if (w == M) {
            if (threadIdx.x == 0) {
                a.status[0] = M + 1;
                a.status[1] = i;
            }
            return;
        }
        __syncthreads();   // pts and qc are rewritten for the next solution
    }
}

__global__ void __launch_bounds__(kTrackThreads) k_track(TrackArgs a) { track_body(a); }

// Many queries in one launch: block b tracks query b, its arguments copied to LDS.
__global__ void __launch_bounds__(kTrackThreads) k_track_batch(const TrackArgs* __restrict__ args) {
    __shared__ TrackArgs a;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(args + blockIdx.x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&a);
    for (uint32_t i = threadIdx.x; i < sizeof(TrackArgs) / 4; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    track_body(a);
}

hipError_t launch_track(const TrackArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_track, dim3(1), dim3(kTrackThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_track_batch(const TrackArgs* args, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_track_batch, dim3((uint32_t)count), dim3(kTrackThreads), 0, st, args);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tube path search ("Smooth sequence computation", "Filtering for smoothness").
// Waypoint w has the frame g_w - r .. g_w + r per joint, g_w the guide
// start + round_half_away(w*(goal - start)/W); cell digits are base 2r+1 with joint 0
// most significant, so the cell index orders poses lexicographically.
// ---------------------------------------------------------------------------
// 32-bit arithmetic is exact here: W <= 4096 and |goal - start| < 2 * 256 steps, so
// 2 |w (goal - start)| + W < 2^31 (the host rejects larger W).
__device__ __forceinline__ int guide_at(const TubeArgs& a, const int* goal, int w, int k) {
    const int num = w * (goal[k] - a.start[k]);
    const uint32_t mag = (2u * (uint32_t)(num < 0 ? -num : num) + (uint32_t)a.W) / (2u * (uint32_t)a.W);
    return a.start[k] + (num < 0 ? -(int)mag : (int)mag);
}


// Tube validity by prefix.  A thread takes one pose prefix (joints 0 .. n-L-1) of one
// waypoint frame, replays it once, then tries the B^L completions of the last L joints
// (L <= 2), so that a segment shared by many cells is tested once.  A cell is valid
// when every joint is in its range (the start pose at waypoint 0, the reach pose at
// waypoint W) and the replay of the pose is clear.  Output: bytes, or bits OR-ed into a
// zeroed bitset (completions of one prefix are consecutive cells).
__device__ __forceinline__ bool tube_angle(const TubeArgs& a, const int* goal, int w, int k, int d, int& q) {
    q = guide_at(a, goal, w, k) - a.r + d;
    if (w == 0) return q == a.start[k];
    if (w == a.W) return q == goal[k];
    return q >= a.lim_lo[k] && q <= a.lim_hi[k];
}

struct FkState {
    int x, y, z, ia, ie;
};

__device__ __forceinline__ bool fk_step(const TubeArgs& a, int k, int qk, FkState& s) {
    const JointView& J = a.joints[k];
    if (J.type == 0)
        s.ia = wrap_na(s.ia + qk, a.na);
    else
        s.ie = wrap_na(s.ie + qk, a.na);
    const int o = s.ia * a.na + s.ie;
    const bool ok = segment_clear_all(a.g, J, o, s.x, s.y, s.z);
    const short4 d = J.off[o];
    s.x += d.x;
    s.y += d.y;
    s.z += d.z;
    return ok;
}

// With `goals` (attempt-major, n values each) the grid's y index is an attempt: its goal
// replaces a.goal and its frames lie vstride words further in vbits.
__global__ void k_tube_valid_tree(TubeArgs a, int L, uint8_t* vbytes, uint64_t* vbits, TubeBlk tb,
                                  const int32_t* goals, uint64_t vstride) {
    const int n = a.n, B = 2 * a.r + 1, np = n - L;
    __shared__ int goal[kMaxDof];
    if ((int)threadIdx.x < n) goal[threadIdx.x] = goals ? goals[blockIdx.y * n + threadIdx.x] : a.goal[threadIdx.x];
    __syncthreads();
    if (goals) vbits += blockIdx.y * vstride;
    uint32_t P = 1, BL = 1;
    for (int k = 0; k < np; ++k) P *= (uint32_t)B;
    for (int k = 0; k < L; ++k) BL *= (uint32_t)B;
    const uint64_t total = (uint64_t)(a.W + 1) * P;
    for (uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        const int w = (int)(idx / P);
        const uint32_t pre = (uint32_t)(idx - (uint64_t)w * P);
        FkState s{a.bx, a.by, a.bz, a.ia0, a.ie0};
        bool ok = cell_free(a.g, s.x, s.y, s.z);
        uint32_t rest = pre, div = P;
        for (int k = 0; k < np && ok; ++k) {
            div /= (uint32_t)B;
            const int d = (int)(rest / div);
            rest -= (uint32_t)d * div;
            int qk;
            ok = tube_angle(a, goal, w, k, d, qk) && fk_step(a, k, qk, s);
        }
        uint32_t bits = 0;   // bit l: completion l (BL <= 32)
        if (ok) {
            if (L == 0) {
                bits = 1;
            } else if (L == 1) {
                for (int d = 0; d < B; ++d) {
                    FkState t = s;
                    int qk;
                    if (tube_angle(a, goal, w, n - 1, d, qk) && fk_step(a, n - 1, qk, t)) bits |= 1u << d;
                }
            } else {
                for (int d1 = 0; d1 < B; ++d1) {
                    FkState t = s;
                    int q1;
                    if (!(tube_angle(a, goal, w, n - 2, d1, q1) && fk_step(a, n - 2, q1, t))) continue;
                    for (int d2 = 0; d2 < B; ++d2) {
                        FkState u = t;
                        int q2;
                        if (tube_angle(a, goal, w, n - 1, d2, q2) && fk_step(a, n - 1, q2, u))
                            bits |= 1u << (d1 * B + d2);
                    }
                }
            }
        }
        const uint64_t cell0 = (uint64_t)pre * BL;
        if (vbytes) {
            uint8_t* out = vbytes + (uint64_t)w * a.slab + cell0;
            for (uint32_t l = 0; l < BL; ++l) out[l] = (uint8_t)((bits >> l) & 1u);
        } else if (bits) {
            // blocked layout: cell c is bit (c / Bq) 64 b + c % Bq of its frame (L <= q, so
            // the completions of one prefix lie in one block)
            const uint32_t blk = (uint32_t)cell0 / tb.Bq;
            const uint32_t v0 = (uint32_t)cell0 - blk * tb.Bq;
            const uint64_t pos = ((uint64_t)w * tb.nw + (uint64_t)blk * tb.b) * 64 + v0;
            const uint64_t word = pos >> 6;
            const int sh = (int)(pos & 63);
            atomicOr((unsigned long long*)&vbits[word], (unsigned long long)((uint64_t)bits << sh));
            if (sh + (int)BL > 64) atomicOr((unsigned long long*)&vbits[word + 1], (unsigned long long)((uint64_t)bits >> (64 - sh)));
        }
    }
}

uint64_t tube_prefix_threads(const TubeArgs& a, int L);

// Completions per thread: one joint keeps the per-thread chain of segment tests short
// (small frames are latency-bound); two joints halve the segment tests when the frame
// count alone fills the device.
int tube_leaf_joints(const TubeArgs& a) {
    const int B = 2 * a.r + 1;
    if (a.n >= 2 && B * B <= 32 && tube_prefix_threads(a, 1) > (2ull << 20)) return 2;
    if (a.n >= 1 && B <= 32) return 1;
    return 0;
}

uint64_t tube_prefix_threads(const TubeArgs& a, int L) {
    uint64_t P = 1;
    for (int k = 0; k < a.n - L; ++k) P *= (uint64_t)(2 * a.r + 1);
    return (uint64_t)(a.W + 1) * P;
}


hipError_t launch_tube_valid(const TubeArgs& a, uint8_t* valid, hipStream_t st) {
    const int L = tube_leaf_joints(a);
    hipLaunchKernelGGL(k_tube_valid_tree, dim3(grid_for(tube_prefix_threads(a, L))), dim3(kBlock), 0, st, a, L, valid,
                       (uint64_t*)nullptr, TubeBlk{}, (const int32_t*)nullptr, 0ull);
    return hipGetLastError();
}

constexpr int kTubeThreads = 1024;
constexpr uint32_t kSmallSlab = 8192;

// Dilation of one frame cell along joint k: R(c) = OR over e in [-delta, delta] of the
// source cell whose digit k is d + shift + e (the previous frame is shifted by
// `shift` = g_w[k] - g_{w-1}[k] against the current one).
__device__ __forceinline__ uint8_t dilate_cell(const uint8_t* src, uint32_t c, uint32_t stride, int B, int shift,
                                               int delta) {
    int d = (int)((c / stride) % (uint32_t)B);
    uint8_t any = 0;
    for (int e = -delta; e <= delta && !any; ++e) {
        int dp = d + shift + e;
        if (dp < 0 || dp >= B) continue;
        any = src[(int64_t)c + (int64_t)(dp - d) * (int64_t)stride];
    }
    return any;
}

__device__ __forceinline__ void tube_strides(const TubeArgs& a, uint32_t* stride) {
    uint32_t s = 1;
    for (int k = a.n - 1; k >= 0; --k) {
        stride[k] = s;
        s *= (uint32_t)(2 * a.r + 1);
    }
}

// Backward choice ("Smooth sequence computation": work backward from the reach pose,
// at each waypoint the solution closest in configuration to the one found): among the
// reachable poses of frame w-1 within delta of the current pose, the one with the
// smallest L1 distance to the guide, ties by the smallest pose (= smallest cell).
// Runs in one block; `frame0` is frame 0's array, `reach` the frames 1..W.
__device__ void tube_trace_block(const TubeArgs& a, const uint8_t* frame0, const uint8_t* reach, int32_t* path,
                                 int32_t* status, const uint32_t* dig) {
    __shared__ unsigned long long best_part[kTubeThreads / 64];
    __shared__ int qcur[kMaxDof];
    __shared__ int flo[kMaxDof];   // frame origin g_{w-1} - r of the waypoint being chosen
    __shared__ uint32_t stride[kMaxDof];
    __shared__ int fail;
    const int tid = threadIdx.x;
    const int B = 2 * a.r + 1;
    const uint32_t slab = (uint32_t)a.slab;
    if (tid == 0) {
        tube_strides(a, stride);
        fail = 0;
    }
    if (tid < a.n) {
        qcur[tid] = a.goal[tid];
        path[a.W * a.n + tid] = a.goal[tid];
    }
    __syncthreads();
    // candidates: the (2 delta + 1)^n box around the current pose, or the whole frame
    uint64_t ncand = 1;
    for (int k = 0; k < a.n && ncand <= slab; ++k) ncand *= (uint64_t)(2 * a.delta + 1);
    const bool by_box = ncand <= slab && !dig;
    if (!by_box) ncand = slab;
    const uint32_t span = (uint32_t)(2 * a.delta + 1);
    for (int w = a.W; w >= 1; --w) {
        const uint8_t* R = (w - 1 == 0) ? frame0 : reach + (uint64_t)(w - 1) * slab;
        if (tid < a.n) flo[tid] = guide_at(a, a.goal, w - 1, tid) - a.r;
        __syncthreads();
        unsigned long long best = ~0ull;
        for (uint32_t t = tid; t < ncand; t += blockDim.x) {
            uint32_t cell = 0;
            int l1 = 0;
            bool ok = true;
            uint32_t rest = t;
            for (int k = a.n - 1; k >= 0; --k) {
                int d;
                if (by_box) {
                    uint32_t q = rest / span;
                    int e = (int)(rest - q * span) - a.delta;
                    rest = q;
                    d = qcur[k] + e - flo[k];
                    if (d < 0 || d >= B) ok = false;
                } else {
                    if (dig) {
                        d = B == 1 ? 0 : (int)((dig[t] >> (4 * k)) & 15u);
                    } else {
                        uint32_t q = rest / (uint32_t)B;
                        d = (int)(rest - q * (uint32_t)B);
                        rest = q;
                    }
                    int dq = flo[k] + d - qcur[k];
                    if (dq < -a.delta || dq > a.delta) ok = false;
                }
                cell += (uint32_t)(d < 0 ? 0 : d) * stride[k];
                l1 += abs(d - a.r);   // |q - g| with q = g - r + d
            }
            if (!ok || !R[cell]) continue;
            unsigned long long key = ((unsigned long long)l1 << 40) | cell;
            best = key < best ? key : best;
        }
        for (int off = 32; off > 0; off >>= 1) {
            unsigned long long o = __shfl_xor(best, off, 64);
            best = o < best ? o : best;
        }
        if ((tid & 63) == 0) best_part[tid >> 6] = best;
        __syncthreads();
        if (tid == 0) {
            unsigned long long b = ~0ull;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) b = best_part[i] < b ? best_part[i] : b;
            if (b == ~0ull) {
                fail = 1;
            } else {
                uint32_t c = (uint32_t)(b & ((1ull << 40) - 1));
                for (int k = a.n - 1; k >= 0; --k) {
                    int d = (int)(c % (uint32_t)B);
                    c /= (uint32_t)B;
                    qcur[k] = flo[k] + d;
                    path[(w - 1) * a.n + k] = qcur[k];
                }
            }
        }
        __syncthreads();
        if (fail) break;
    }
    if (tid == 0) *status = fail ? 0 : 1;
}

// Small frames: the whole dynamic program in one block, working arrays in LDS.
// R_0 = {start}; R_w = valid_w AND (R_{w-1} dilated by delta in every joint, moved from
// frame w-1 to frame w one joint at a time); frames 1..W are kept for the choice.
__global__ void __launch_bounds__(kTubeThreads) k_tube_small(TubeArgs a, const uint8_t* valid, uint8_t* reach,
                                                             int32_t* path, int32_t* status) {
    __shared__ uint8_t A[kSmallSlab], T0[kSmallSlab], T1[kSmallSlab];
    __shared__ uint32_t dig[kSmallSlab];   // digits of every cell, 4 bits per joint
    __shared__ uint32_t stride[kMaxDof];
    const int tid = threadIdx.x;
    const int B = 2 * a.r + 1;
    const uint32_t slab = (uint32_t)a.slab;
    if (tid == 0) tube_strides(a, stride);
    for (uint32_t c = tid; c < slab; c += blockDim.x) {
        A[c] = valid[c];
        uint32_t packed = 0, rest = c;
        if (B > 1) {
            for (int k = a.n - 1; k >= 0; --k) {
                packed |= (rest % (uint32_t)B) << (4 * k);
                rest /= (uint32_t)B;
            }
        }
        dig[c] = packed;
    }
    __syncthreads();
    for (int w = 1; w <= a.W; ++w) {
        const uint8_t* vw = valid + (uint64_t)w * slab;
        for (int k = 0; k < a.n; ++k) {
            const uint8_t* src = (k == 0) ? A : ((k & 1) ? T0 : T1);
            uint8_t* dst = (k == a.n - 1) ? A : ((k & 1) ? T1 : T0);
            const int shift = guide_at(a, a.goal, w, k) - guide_at(a, a.goal, w - 1, k);
            // the last pass writes A in place of R_{w-1}: read every source cell of
            // this pass before any thread writes
            constexpr int kPer = (kSmallSlab + kTubeThreads - 1) / kTubeThreads;
            uint8_t vals[kPer];
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                uint32_t c = tid + (uint32_t)i * kTubeThreads;
                uint8_t any = 0;
                if (c < slab) {
                    const int d = B == 1 ? 0 : (int)((dig[c] >> (4 * k)) & 15u);
                    for (int e = -a.delta; e <= a.delta && !any; ++e) {
                        int dp = d + shift + e;
                        if (dp < 0 || dp >= B) continue;
                        any = src[(int)c + (dp - d) * (int)stride[k]];
                    }
                    if (k == a.n - 1) any = any && vw[c];
                }
                vals[i] = any;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                uint32_t c = tid + (uint32_t)i * kTubeThreads;
                if (c < slab) dst[c] = vals[i];
            }
            __syncthreads();
        }
        uint8_t* rw = reach + (uint64_t)w * slab;
        for (uint32_t c = tid; c < slab; c += blockDim.x) rw[c] = A[c];
        __syncthreads();
    }
    // goal cell: every digit = r (the guide at w = W is the goal)
    uint32_t gcell = 0;
    for (int k = 0; k < a.n; ++k) gcell += (uint32_t)a.r * stride[k];
    if (!A[gcell]) {
        if (tid == 0) *status = 0;
        return;
    }
    tube_trace_block(a, valid, reach, path, status, dig);
}

// Large frames: one pass of one joint over the whole frame, many blocks.
__global__ void k_tube_pass(TubeArgs a, int w, int k, const uint8_t* src, uint8_t* dst, const uint8_t* valid_w) {
    const int B = 2 * a.r + 1;
    uint32_t stride = 1;
    for (int j = a.n - 1; j > k; --j) stride *= (uint32_t)B;
    const int shift = guide_at(a, a.goal, w, k) - guide_at(a, a.goal, w - 1, k);
    const uint32_t slab = (uint32_t)a.slab;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < slab; c += gridDim.x * blockDim.x) {
        uint8_t any = dilate_cell(src, c, stride, B, shift, a.delta);
        if (valid_w) any = any && valid_w[c];
        dst[c] = any;
    }
}

__global__ void __launch_bounds__(kTubeThreads) k_tube_trace(TubeArgs a, const uint8_t* valid, const uint8_t* reach,
                                                             int32_t* path, int32_t* status) {
    uint32_t gcell = 0, s = 1;
    for (int k = a.n - 1; k >= 0; --k) {
        gcell += (uint32_t)a.r * s;
        s *= (uint32_t)(2 * a.r + 1);
    }
    if (!reach[(uint64_t)a.W * a.slab + gcell]) {
        if (threadIdx.x == 0) *status = 0;
        return;
    }
    tube_trace_block(a, valid, reach, path, status, nullptr);
}

// ---------------------------------------------------------------------------
// Bit-parallel tube search.  A frame is a bitset in a blocked layout: the last q joints
// (inner, B^q <= 128 cells) form a block of b = 1 or 2 words; cell (u, v), u the index
// of the outer digits and v of the inner ones, is bit u*64b + v.  Along an outer joint
// a shift by t cells is a move of whole blocks, kept where the block's digit stays in
// range (digits from a table in LDS); along an inner joint it is a shift inside the
// block, masked by a pattern that every block shares.  Two frames alternate in LDS; the
// reachable sets R_w go to global memory for the backward choice.  One block runs the
// whole dynamic program.
// ---------------------------------------------------------------------------
constexpr int kBlkThreads = 1024;
constexpr int kBlkMaxB = 11;                  // frame edge 2r+1 (r <= 5)
constexpr int kBlkPatterns = 24;              // q (B + 1) digit-at-least patterns
constexpr int kBlkLevels = 16;                // inner L1 levels q r + 1
constexpr size_t kBlkLdsMax = 150 * 1024;     // dynamic LDS (a CU has 160 KiB)

__host__ __device__ inline size_t align8(size_t v) { return (v + 7) & ~(size_t)7; }

TubeBlk tube_blk_plan(const TubeArgs& a) {
    TubeBlk t{};
    const int B = 2 * a.r + 1;
    if (a.n < 1 || B > kBlkMaxB) return t;
    int q = 0;
    uint32_t Bq = 1;
    while (q < a.n && Bq * (uint32_t)B <= 128u) {
        Bq *= (uint32_t)B;
        ++q;
    }
    if (q < 1 || q * (B + 1) > kBlkPatterns || q * a.r + 1 > kBlkLevels) return t;
    uint64_t nblk = 1;
    for (int k = 0; k < a.n - q; ++k) {
        nblk *= (uint64_t)B;
        if (nblk > (1u << 20)) return TubeBlk{};
    }
    t.q = q;
    t.no = a.n - q;
    t.Bq = Bq;
    t.b = Bq > 64 ? 2 : 1;
    t.nblk = (uint32_t)nblk;
    t.nw = nblk * (uint64_t)t.b;
    const size_t bytes = 2 * t.nw * 8 + align8(nblk * (uint64_t)t.no) + align8(nblk);
    t.lds = bytes <= kBlkLdsMax ? bytes : 0;
    // small frames: every validity and reach frame stays in LDS, so no waypoint waits
    // on a global memory round trip
    const size_t frames = 2 * (size_t)(a.W + 1) * t.nw * 8;
    if (t.lds && bytes + frames <= kBlkLdsMax) {
        t.frames_lds = 1;
        t.lds = bytes + frames;
    }
    return t;
}

// (x1:x0) >> s and << s for 0 <= s < 128
__device__ __forceinline__ void shr128(uint64_t x0, uint64_t x1, int s, uint64_t& y0, uint64_t& y1) {
    if (s == 0) {
        y0 = x0;
        y1 = x1;
    } else if (s < 64) {
        y0 = (x0 >> s) | (x1 << (64 - s));
        y1 = x1 >> s;
    } else {
        y0 = x1 >> (s - 64);
        y1 = 0;
    }
}

__device__ __forceinline__ void shl128(uint64_t x0, uint64_t x1, int s, uint64_t& y0, uint64_t& y1) {
    if (s == 0) {
        y0 = x0;
        y1 = x1;
    } else if (s < 64) {
        y0 = x0 << s;
        y1 = (x1 << s) | (x0 >> (64 - s));
    } else {
        y0 = 0;
        y1 = x0 << (s - 64);
    }
}

template <int DL, bool FL>
__global__ void __launch_bounds__(kBlkThreads) k_tube_blk(TubeArgs a, TubeBlk tb, const uint64_t* vbits,
                                                          uint64_t* rbits, int32_t* path, int32_t* status,
                                                          const int32_t* goals, uint64_t vstride) {
    // with `goals`, block i searches attempt i: its goal, frames vstride words further,
    // its own path rows and status
    if (goals) {
        const uint64_t att = blockIdx.x;
        vbits += att * vstride;
        rbits += att * vstride;
        path += att * (uint64_t)(a.W + 1) * a.n;
        status += att;
    }
    extern __shared__ uint64_t sm[];
    const int n = a.n, B = 2 * a.r + 1, r = a.r, dl = DL > 0 ? DL : a.delta;
    const int no = tb.no, q = tb.q, b = tb.b;
    const uint32_t nblk = tb.nblk, Bq = tb.Bq;
    const int nw = (int)tb.nw;
    const size_t nfw = FL ? (size_t)(a.W + 1) * nw : 0;            // words of the LDS frames
    uint64_t* fa = sm;
    uint64_t* fb = sm + nw;
    const uint64_t* V = FL ? sm + 2 * nw : vbits;                  // validity frames
    uint64_t* R = FL ? sm + 2 * nw + nfw : rbits;                  // reach frames
    uint8_t* dig = reinterpret_cast<uint8_t*>(sm + 2 * nw + 2 * nfw);  // [block][outer joint]
    uint8_t* l1o = dig + align8((size_t)nblk * no);                // outer L1 distance per block
    __shared__ uint32_t sblk[kMaxDof], scell[kMaxDof];
    __shared__ unsigned long long pge[kBlkPatterns * 2];           // [inner joint][v <= B][word]
    __shared__ unsigned long long plv[kBlkLevels * 2];             // [inner L1 level][word]
    __shared__ int shw[kMaxDof], dlo[kMaxDof], dhi[kMaxDof], flo[kMaxDof], qcur[kMaxDof];
    __shared__ unsigned long long best_part[kBlkThreads / 64];
    __shared__ int fail;
    __shared__ int gstart[kMaxDof], gdiff[kMaxDof];     // the guide's ends, read once
    // guide_at from the LDS copy (the argument block is not re-read in the serial loops)
    auto sguide = [&](int w, int k) {
        const int num = w * gdiff[k];
        const uint32_t mag = (2u * (uint32_t)(num < 0 ? -num : num) + (uint32_t)a.W) / (2u * (uint32_t)a.W);
        return gstart[k] + (num < 0 ? -(int)mag : (int)mag);
    };
    const int tid = threadIdx.x;
    const int nthr = (int)blockDim.x;    // a multiple of 64, fewer for small frames
    if (tid == 0) {
        uint32_t st = 1;
        for (int k = n - 1; k >= no; --k) {
            scell[k] = st;
            st *= (uint32_t)B;
        }
        st = 1;
        for (int k = no - 1; k >= 0; --k) {
            sblk[k] = st;
            st *= (uint32_t)B;
        }
        fail = 0;
    }
    if (tid < n) {
        gstart[tid] = a.start[tid];
        gdiff[tid] = (goals ? goals[blockIdx.x * n + tid] : a.goal[tid]) - a.start[tid];
    }
    __syncthreads();
    // inner patterns, one thread per inner cell c: its bit goes into "digit of inner joint
    // ki >= v" for v <= its digit, and into its inner L1 level
    for (int i = tid; i < 2 * (kBlkPatterns + kBlkLevels); i += nthr) {
        if (i < 2 * kBlkPatterns) pge[i] = 0; else plv[i - 2 * kBlkPatterns] = 0;
    }
    __syncthreads();
    for (uint32_t c = tid; c < Bq; c += nthr) {
        const int word = c >> 6;
        const unsigned long long bit = 1ull << (c & 63);
        int d1 = 0;
        for (int ki = 0; ki < q; ++ki) {
            const int d = (int)((c / scell[no + ki]) % (uint32_t)B);
            d1 += d > r ? d - r : r - d;
            for (int v = 0; v <= d; ++v) atomicOr(&pge[(ki * (B + 1) + v) * 2 + word], bit);
        }
        atomicOr(&plv[d1 * 2 + word], bit);
    }
    // outer digits and L1 distance per block; R_0 = {start}
    for (uint32_t u = tid; u < nblk; u += nthr) {
        int d1 = 0;
        for (int k = 0; k < no; ++k) {
            const int d = (int)((u / sblk[k]) % (uint32_t)B);
            dig[(size_t)u * no + k] = (uint8_t)d;
            d1 += d > r ? d - r : r - d;
        }
        l1o[u] = (uint8_t)d1;
    }
    if constexpr (FL) {
        for (size_t i = tid; i < nfw; i += nthr) sm[2 * nw + i] = vbits[i];
        __syncthreads();
    }
    for (int i = tid; i < nw; i += nthr) {
        fa[i] = V[i];
        R[i] = V[i];
    }
    __syncthreads();
    // Forward: R_w = valid_w AND the delta-dilation of R_{w-1}.  The dilation is a
    // product over joints, so its order is free: the outer joints move whole blocks (one
    // pass each, through LDS), then each thread dilates its own blocks along the inner
    // joints in registers and applies the validity frame.
    uint64_t* src = fa;
    uint64_t* dst = fb;
    for (int w = 1; w <= a.W; ++w) {
        if (tid < n) shw[tid] = sguide(w, tid) - sguide(w - 1, tid);
        __syncthreads();
        for (int k = 0; k < no; ++k) {
            const int sh = shw[k];
            // outer joint: whole blocks move by t * S blocks
            const int S = (int)sblk[k];
            for (uint32_t u = tid; u < nblk; u += nthr) {
                const int d = dig[(size_t)u * no + k];
                uint64_t a0 = 0, a1 = 0;
                auto take = [&](int e) {
                    const int t = sh + e;
                    if (d + t < 0 || d + t >= B) return;
                    const size_t from = ((size_t)u + (ptrdiff_t)t * S) * (size_t)b;
                    a0 |= src[from];
                    if (b == 2) a1 |= src[from + 1];
                };
                if constexpr (DL > 0) {
#pragma unroll
                    for (int e = -DL; e <= DL; ++e) take(e);
                } else {
                    for (int e = -dl; e <= dl; ++e) take(e);
                }
                dst[(size_t)u * b] = a0;
                if (b == 2) dst[(size_t)u * b + 1] = a1;
            }
            __syncthreads();
            uint64_t* tmp = src;
            src = dst;
            dst = tmp;
        }
        // inner joints: shifts by t * s cells inside the block, in registers
        for (uint32_t u = tid; u < nblk; u += nthr) {
            const size_t i0 = (size_t)u * b;
            uint64_t x0 = src[i0], x1 = b == 2 ? src[i0 + 1] : 0ull;
            for (int ki = 0; ki < q; ++ki) {
                const int sh = shw[no + ki];
                const int s1 = (int)scell[no + ki];
                uint64_t a0 = 0, a1 = 0;
                auto take = [&](int e) {
                    const int t = sh + e;
                    const int vlo = t < 0 ? -t : 0;
                    const int vend = t > 0 ? B - t : B;        // exclusive
                    if (vlo >= vend) return;
                    const int lo_i = (ki * (B + 1) + vlo) * 2, hi_i = (ki * (B + 1) + vend) * 2;
                    const uint64_t m0 = pge[lo_i] & ~pge[hi_i], m1 = pge[lo_i + 1] & ~pge[hi_i + 1];
                    uint64_t y0, y1;
                    if (t >= 0)
                        shr128(x0, x1, t * s1, y0, y1);
                    else
                        shl128(x0, x1, -t * s1, y0, y1);
                    a0 |= y0 & m0;
                    a1 |= y1 & m1;
                };
                if constexpr (DL > 0) {
#pragma unroll
                    for (int e = -DL; e <= DL; ++e) take(e);
                } else {
                    for (int e = -dl; e <= dl; ++e) take(e);
                }
                x0 = a0;
                x1 = a1;
            }
            const size_t g0 = (size_t)w * nw + i0;
            x0 &= V[g0];
            R[g0] = x0;
            dst[i0] = x0;
            if (b == 2) {
                x1 &= V[g0 + 1];
                R[g0 + 1] = x1;
                dst[i0 + 1] = x1;
            }
        }
        __syncthreads();
        uint64_t* tmp = src;
        src = dst;
        dst = tmp;
    }
    // the goal: every digit = r
    {
        uint32_t ug = 0, vg = 0;
        for (int k = 0; k < no; ++k) ug += (uint32_t)r * sblk[k];
        for (int k = no; k < n; ++k) vg += (uint32_t)r * scell[k];
        const uint64_t word = src[(size_t)ug * b + (vg >> 6)];
        if (!((word >> (vg & 63)) & 1ull)) {
            if (tid == 0) *status = 0;
            return;
        }
    }
    if (tid < n) {
        qcur[tid] = gstart[tid] + gdiff[tid];
        path[a.W * n + tid] = qcur[tid];
    }
    // Backward choice: among the reachable cells of frame w-1 whose digits lie within
    // delta of the current pose, the smallest L1 distance to the guide, ties by the
    // smallest cell (u Bq + v orders poses lexicographically).
    for (int w = a.W; w >= 1; --w) {
        if (tid < n) {
            const int f = sguide(w - 1, tid) - r;
            const int lo = qcur[tid] - dl - f, hi = qcur[tid] + dl - f;
            flo[tid] = f;
            dlo[tid] = lo < 0 ? 0 : lo;
            dhi[tid] = hi > B - 1 ? B - 1 : hi;
        }
        __syncthreads();
        uint64_t ib0 = Bq >= 64 ? ~0ull : ((1ull << Bq) - 1);
        uint64_t ib1 = Bq > 64 ? (Bq >= 128 ? ~0ull : ((1ull << (Bq - 64)) - 1)) : 0ull;
        for (int ki = 0; ki < q; ++ki) {
            const int lo = dlo[no + ki], he = dhi[no + ki] + 1;
            if (lo >= he) {
                ib0 = ib1 = 0;
                break;
            }
            const int lo_i = (ki * (B + 1) + lo) * 2, hi_i = (ki * (B + 1) + he) * 2;
            ib0 &= pge[lo_i] & ~pge[hi_i];
            ib1 &= pge[lo_i + 1] & ~pge[hi_i + 1];
        }
        const uint64_t* Rw = R + (size_t)(w - 1) * nw;
        unsigned long long best = ~0ull;
        if (ib0 | ib1) {
            for (uint32_t u = tid; u < nblk; u += nthr) {
                bool in = true;
                for (int k = 0; k < no; ++k) {
                    const int d = dig[(size_t)u * no + k];
                    in = in && d >= dlo[k] && d <= dhi[k];
                }
                if (!in) continue;
                const uint64_t m0 = Rw[(size_t)u * b] & ib0;
                const uint64_t m1 = b == 2 ? (Rw[(size_t)u * b + 1] & ib1) : 0ull;
                if (!(m0 | m1)) continue;
                const unsigned long long lo1 = l1o[u];
                for (int l = 0; l <= q * r; ++l) {
                    const uint64_t h0 = m0 & plv[l * 2], h1 = m1 & plv[l * 2 + 1];
                    if (h0 | h1) {
                        const uint32_t v = h0 ? (uint32_t)(__ffsll((unsigned long long)h0) - 1)
                                              : 64u + (uint32_t)(__ffsll((unsigned long long)h1) - 1);
                        const unsigned long long key = ((lo1 + (unsigned long long)l) << 40) |
                                                       ((unsigned long long)u * Bq + v);
                        best = key < best ? key : best;
                        break;
                    }
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(best, off, 64);
            best = o < best ? o : best;
        }
        if ((tid & 63) == 0) best_part[tid >> 6] = best;
        __syncthreads();
        if (tid < n) {
            unsigned long long bb = ~0ull;
            for (int i = 0; i < nthr / 64; ++i) bb = best_part[i] < bb ? best_part[i] : bb;
            if (bb == ~0ull) {
                if (tid == 0) fail = 1;
            } else {
                const uint32_t c = (uint32_t)(bb & ((1ull << 40) - 1));
                const uint32_t u = c / Bq, v = c - u * Bq;
                const int d = tid < no ? (int)dig[(size_t)u * no + tid] : (int)((v / scell[tid]) % (uint32_t)B);
                qcur[tid] = flo[tid] + d;
                path[(w - 1) * n + tid] = qcur[tid];
            }
        }
        __syncthreads();
        if (fail) break;
    }
    if (tid == 0) *status = fail ? 0 : 1;
}

template <int DL, bool FL>
hipError_t launch_tube_blk_dl(const TubeArgs& a, const TubeBlk& t, const uint64_t* vbits, uint64_t* rbits,
                              int32_t* path, int32_t* status, hipStream_t st, int A, const int32_t* goals,
                              uint64_t vstride) {
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
        attr = hipFuncSetAttribute((const void*)k_tube_blk<DL, FL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kBlkLdsMax);
    });
    if (attr != hipSuccess) return attr;
    // threads: one per block of the frame, rounded to waves (barriers of idle waves cost)
    const uint32_t threads = std::min<uint32_t>(kBlkThreads, std::max<uint32_t>(64u, (t.nblk + 63u) & ~63u));
    hipLaunchKernelGGL((k_tube_blk<DL, FL>), dim3(A), dim3(threads), t.lds, st, a, t, vbits, rbits, path, status,
                       goals, vstride);
    return hipGetLastError();
}

template <int DL>
hipError_t launch_tube_blk_dl(const TubeArgs& a, const TubeBlk& t, const uint64_t* vbits, uint64_t* rbits,
                              int32_t* path, int32_t* status, hipStream_t st, int A, const int32_t* goals,
                              uint64_t vstride) {
    if (t.frames_lds) return launch_tube_blk_dl<DL, true>(a, t, vbits, rbits, path, status, st, A, goals, vstride);
    return launch_tube_blk_dl<DL, false>(a, t, vbits, rbits, path, status, st, A, goals, vstride);
}

hipError_t launch_tube_bits(const TubeArgs& a, const TubeBlk& t, uint64_t* vbits, uint64_t* rbits, int32_t* path,
                            int32_t* status, hipStream_t st, int A, const int32_t* goals) {
    if (A < 1 || (A > 1 && !goals) || A > 65535) return hipErrorInvalidValue;
    const int L = std::min(tube_leaf_joints(a), t.q);
    const uint64_t stride = (uint64_t)(a.W + 1) * t.nw;   // words of one attempt's frames
    hipError_t e = launch_fill(vbits, (uint64_t)A * stride, 0ull, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tube_valid_tree, dim3(grid_for(tube_prefix_threads(a, L)), A), dim3(kBlock), 0, st, a, L,
                       (uint8_t*)nullptr, vbits, t, goals, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.delta == 1) return launch_tube_blk_dl<1>(a, t, vbits, rbits, path, status, st, A, goals, stride);
    if (a.delta == 2) return launch_tube_blk_dl<2>(a, t, vbits, rbits, path, status, st, A, goals, stride);
    return launch_tube_blk_dl<0>(a, t, vbits, rbits, path, status, st, A, goals, stride);
}

hipError_t launch_tube_solve(const TubeArgs& a, const uint8_t* valid, uint8_t* reach, uint8_t* tmp0,
                             uint8_t* tmp1, int32_t* path, int32_t* status, hipStream_t st) {
    if (a.slab <= kSmallSlab) {
        hipLaunchKernelGGL(k_tube_small, dim3(1), dim3(kTubeThreads), 0, st, a, valid, reach, path, status);
        return hipGetLastError();
    }
    const uint32_t blocks = grid_for(a.slab);
    for (int w = 1; w <= a.W; ++w) {
        const uint8_t* prev = (w == 1) ? valid : reach + (uint64_t)(w - 1) * a.slab;
        for (int k = 0; k < a.n; ++k) {
            const uint8_t* src = (k == 0) ? prev : ((k & 1) ? tmp0 : tmp1);
            uint8_t* dst = (k == a.n - 1) ? reach + (uint64_t)w * a.slab : ((k & 1) ? tmp1 : tmp0);
            const uint8_t* vw = (k == a.n - 1) ? valid + (uint64_t)w * a.slab : nullptr;
            hipLaunchKernelGGL(k_tube_pass, dim3(blocks), dim3(kBlock), 0, st, a, w, k, src, dst, vw);
        }
    }
    hipLaunchKernelGGL(k_tube_trace, dim3(1), dim3(kTubeThreads), 0, st, a, valid, reach, path, status);
    return hipGetLastError();
}

}  // namespace msc
