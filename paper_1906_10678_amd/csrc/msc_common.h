// Internal types shared by the HIP kernels and the host runtime of libmsc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msc {

constexpr int kMaxDof = 16;
constexpr int kMaxNa = 256;
constexpr uint64_t kEmpty = ~0ull;        // free hash slot
constexpr uint64_t kDead = 1ull << 63;    // hash entry removed from the set (key kept)

// Internal state key: x | y << 10 | z << 20 | ia << 32 | ie << 40 (grids up to 1024^3).
__host__ __device__ inline uint64_t pack_key(int x, int y, int z, int ia, int ie) {
    return (uint64_t)(uint32_t)x | ((uint64_t)(uint32_t)y << 10) | ((uint64_t)(uint32_t)z << 20) |
           ((uint64_t)(uint32_t)ia << 32) | ((uint64_t)(uint32_t)ie << 40);
}
__host__ __device__ inline void unpack_key(uint64_t k, int& x, int& y, int& z, int& ia, int& ie) {
    x = (int)(k & 1023);
    y = (int)((k >> 10) & 1023);
    z = (int)((k >> 20) & 1023);
    ia = (int)((k >> 32) & 255);
    ie = (int)((k >> 40) & 255);
}

// Bit-packed occupancy: word (z*n + y)*wpr + x/64, bit x%64; 1 = blocked.
struct GridView {
    const uint64_t* occ;
    int n;
    int wpr;
};

// Rounded segment geometry of one joint: off[o] and sweep[o*S + s] (s = 0..S-1 is
// sample s+1 of S), o = ia*na + ie.
struct JointView {
    const short4* off;
    const short4* sweep;
    int type;   // 0 yaw, 1 pitch
    int lo, hi; // joint window in steps
    int S;
};

// A stage set: a dense bitset over a voxel box x all orientations, or an open-addressing
// hash set of keys.
enum { kDense = 0, kHash = 1 };
struct SetView {
    uint64_t* words;  // dense bit words or hash slots
    uint64_t cap;     // number of words / slots (hash: power of two)
    int kind;
    int fast_ia;      // dense: 1 -> orientation index ie*na + ia, 0 -> ia*na + ie
    int na;
    int x0, y0, z0, nx, ny, nz;  // dense box
};

__host__ __device__ inline uint64_t mix64(uint64_t v) {
    v ^= v >> 33;
    v *= 0xff51afd7ed558ccdull;
    v ^= v >> 33;
    v *= 0xc4ceb9fe1a85ec53ull;
    v ^= v >> 33;
    return v;
}

// Launch shape of the grid-stride set kernels, chosen by the autotuner: the grid cap
// (blocks; more work items per thread below it) and a change of the number of lanes
// that share one state (log2, added to the launch's own choice, clamped to 0..6).
// Every shape gives the same sets: only the mapping of work to threads changes.
struct Shape {
    uint32_t max_blocks = 16384;
    int lg_bias = 0;
};

// Timing of the next set-expansion launch (launch_expand_fwd / launch_expand_bwd) by
// events attached to its dispatch; host thread local.  take_launch_events_used clears
// them and tells whether a launch used them.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool take_launch_events_used();

// Launch wrappers (msc_kernels.hip).  All enqueue on `st`.
hipError_t launch_fill(uint64_t* p, uint64_t n, uint64_t value, hipStream_t st);
hipError_t launch_tables(int na, int S, int L, short4* off, short4* sweep, unsigned int* maxn2,
                         hipStream_t st);
// Obstacle lists carried in the raster kernel's arguments: boxes (lo x, y, z, extent x,
// y, z) then spheres (centre x, y, z, radius), at most kRasterInline values.
constexpr int kRasterInline = 720;
struct RasterInline {
    int32_t v[kRasterInline];
};
hipError_t launch_raster_inline(uint64_t* occ, int n, int wpr, int r, const RasterInline& inl, int nbox, int nsph,
                                hipStream_t st);
hipError_t launch_raster(uint64_t* occ, int n, int wpr, int r, const int32_t* boxes, int nbox,
                         const int32_t* spheres, int nsph, hipStream_t st);
// Moving boxes of one tick, passed by value: (lo x, y, z, ext x, y, z) per box.
constexpr int kDynBoxes = 16;
struct DynBoxes {
    int32_t b[kDynBoxes * 6];
    int count;
};
// dst = src | dilated boxes (src may equal dst).
hipError_t launch_raster_dyn(uint64_t* dst, const uint64_t* src, int n, int wpr, int r, const DynBoxes& db,
                             hipStream_t st);
struct OrientArgs {
    int n, na, ia0, ie0;
    int type[kMaxDof], lo[kMaxDof], hi[kMaxDof];
};
hipError_t launch_orient(const OrientArgs& a, uint64_t* rows_ie, uint64_t* rows_ia, hipStream_t st);
// Copy n counters to (host-mapped) memory with one small kernel.
// flag / seq: see k_publish (flag may be null)
hipError_t launch_publish(const unsigned long long* src, unsigned long long* dst, int n, unsigned long long* flag,
                          unsigned long long seq, hipStream_t st);
// seeds: also write their states to `list` (capacity 1, resp. na^2) and count them;
// cone: approach-cone rows of the final orientation (may be null)
hipError_t launch_seed_fwd(SetView s, GridView g, int x, int y, int z, int ia, int ie, uint64_t* list,
                           unsigned long long* counter, hipStream_t st);
hipError_t launch_seed_bwd(SetView s, GridView g, int x, int y, int z, const uint64_t* rows_ie, int prune,
                           const uint64_t* cone, uint64_t* list, unsigned long long* counter, hipStream_t st);
hipError_t launch_expand_fwd(const uint64_t* in, uint64_t count, SetView out, GridView g, JointView j,
                             int tx, int ty, int tz, long long r2, unsigned long long* counter,
                             unsigned long long* overflow, hipStream_t st, Shape sh = Shape{});
// Zeroes every orientation row of a dense set (fast axis = the joint's) that a backward
// stage from `in` can have written.
// Zeroes the word of every state of a dense set's member list.
hipError_t launch_unlist(const uint64_t* list, uint64_t count, SetView s, hipStream_t st);
hipError_t launch_unexpand_bwd(const uint64_t* in, uint64_t count, SetView out, JointView j, hipStream_t st);
hipError_t launch_expand_bwd(const uint64_t* in, uint64_t count, SetView out, GridView g, JointView j,
                             int bx, int by, int bz, long long r2, const uint64_t* orows,
                             unsigned long long* counter, unsigned long long* overflow,
                             hipStream_t st, Shape sh = Shape{});
// Adds the non-zero words of s (dense: words != 0; hash: slots holding a member) to *counter.
hipError_t launch_count_words(SetView s, unsigned long long* counter, hipStream_t st);
hipError_t launch_compact(SetView s, uint64_t* list, uint64_t cap, unsigned long long* counter,
                          unsigned long long* overflow, hipStream_t st);
hipError_t launch_join(const uint64_t* flist, uint64_t count, SetView f, SetView b,
                       unsigned long long* counter, hipStream_t st);
constexpr int kMeetInsert = 0, kMeetCount = 1, kMeetMark = 2;
// (tx, ty, tz), r2: the target and the squared forward pruning radius of stage m (r2 < 0: none)
hipError_t launch_meet(const uint64_t* flist, uint64_t count, SetView fprev, SetView b, SetView c, GridView g,
                       JointView j, int mode, unsigned long long* c_count, unsigned long long* kept_count,
                       unsigned long long* overflow, int tx, int ty, int tz, long long r2, hipStream_t st,
                       Shape sh = Shape{});
hipError_t launch_dmark(const uint64_t* flist, uint64_t count, SetView fprev, SetView fnext, GridView g,
                        JointView j, unsigned long long* counter, int tx, int ty, int tz, long long r2,
                        hipStream_t st, Shape sh = Shape{});

struct DfsArgs {
    SetView sets[kMaxDof + 1];  // sets[k] = D_k for k <= m, B_k for k > m (k = 0..n)
    JointView joints[kMaxDof];
    GridView g;
    int n, m, na, want;
    int ref[kMaxDof];
    uint64_t root;             // root state key
    int32_t* sols;             // want * n joint values (steps)
    int32_t* nsol;
};
hipError_t launch_dfs(const DfsArgs& a, hipStream_t st);

struct PoseArgs {
    JointView joints[kMaxDof];
    GridView g;
    int n, na, bx, by, bz, ia0, ie0;
};
hipError_t launch_pose_check(const PoseArgs& a, const int32_t* q, int64_t count, uint8_t* valid,
                             int32_t* ends, hipStream_t st);

// Exact end point of discrete poses (FP64): angles in degrees, lengths in voxels.
struct RefineArgs {
    int n;
    int q_div;                 // pose values are divided by this first (1: already in steps)
    int type[kMaxDof];
    double len[kMaxDof];
    double base[3], az0, el0, step;
};
hipError_t launch_refine(const RefineArgs& a, const int32_t* q_steps, const double* targets, int64_t count,
                         double* angles, int32_t* status, hipStream_t st);

// Short-reach shortcut ("Short Reaches").  Hit key of a segment hypothesis: path length
// (1/S voxel) << 40 | squared distance of the hit point << 24 | segment (1-based) << 16.
struct HitArgs {
    GridView g;
    int na;
    int tx, ty, tz;
    int rho2;
    int k;                  // segment (1-based) of the hypotheses
    long long base_len;     // S * (L_1 + ... + L_{k-1})
    int len;                // L_k
};
// Least hit key over F_{k-1}'s states x joint k's window into *best (atomicMin).
hipError_t launch_hits(const uint64_t* in, uint64_t count, JointView j, HitArgs h, unsigned long long* best,
                       hipStream_t st);
// D_{k-1}: removes from fprev the states of its list with no angle whose hit key is *best.
hipError_t launch_hit_mark(const uint64_t* in, uint64_t count, SetView fprev, JointView j, HitArgs h,
                           const unsigned long long* best, hipStream_t st);
struct HitWalkArgs {
    SetView D[kMaxDof];     // D_1 .. D_{k-1} (index j)
    JointView joints[kMaxDof];
    HitArgs h;
    int na, bx, by, bz, ia0, ie0;
    const unsigned long long* best;
    int32_t* out;           // out: k joint values (steps), then the hit sample s (1-based); s = 0: none
};
// The canonical walk from the root into the marked D sets, then the first angle of joint
// k with the best hit (one wave).
hipError_t launch_hit_walk(const HitWalkArgs& a, hipStream_t st);

// The paper's gap search ("The gap in gMS"): quiver vectors (FP64, host-built) for
// segments 1, 2 and 4, a free vector across the gap for segment 3.
struct GmsArgs {
    GridView g;
    const double* Q;        // quiver vectors, 3 per entry
    int nq;
    double L1, L2, L3, L4;
    double p0[3], t[3];
    double ts[64];          // sample fractions s / S, s = 1..S
    int S;
    double min_el;          // sin(least elevation of segment 1) - band
    double c1, c2, c3;      // cos(flexion limits) - band
    double ax[3];           // approach axis (unit), cone_c = cos(half) - band; has_cone = 0: none
    double cone_c;
    int has_cone;
    double r5sq, r7sq;      // squared pruning radii (eqs 5-8, widened by eps)
    double glo, ghi;        // squared bounds of the free vector's length
};
// flags1[i] = 1 when quiver vector i is a segment-1 survivor (Step 1); flags4[l] = 1 when
// it is an admissible, clear segment 4.
hipError_t launch_gms_flags(const GmsArgs& a, uint8_t* flags1, uint8_t* flags4, hipStream_t st);
// The segment-4 list in cluster order (kGmsCluster points per cluster): p3 = t - L4 r_l.
constexpr int kGmsCluster = 16;
struct GmsPoint {
    double x, y, z;
    int32_t l, pad;
};
// A cluster's centre and the squared bounds on |centre - p2| outside which none of its
// points can pass the gap's length test (lo2 < 0: no lower bound).
struct GmsCluster {
    double cx, cy, cz, lo2, hi2, pad;
};
hipError_t launch_gms_points(const GmsArgs& a, const int32_t* order, int n4, GmsPoint* pts, hipStream_t st);
// Steps 2A/2B over (survivor ii, quiver j) pairs, min_ii <= ii <= max_ii, against the
// clustered segment-4 list: per_i[ii] += the solutions of survivor ii; with store, keys
// i << 40 | j << 20 | l are written to slots taken from *slots while they are below cap.
hipError_t launch_gms_pairs(const GmsArgs& a, const int32_t* s1, int n1, const GmsPoint* pts, int n4,
                            const GmsCluster* cl, int ncl, unsigned long long* slots, unsigned long long* per_i,
                            uint64_t* keys, uint64_t cap, int min_ii, int max_ii, int store, hipStream_t st);
// The vectors of solutions keys[n]: 18 doubles each (s1, s2, v3, s4, s3, s4').
hipError_t launch_gms_vectors(const GmsArgs& a, const uint64_t* keys, int n, double* out, hipStream_t st);

// Waypoint tracking of the workspace-guided paths ("Path Planning", "Smooth sequence
// computation", "Filtering for smoothness", "Path between Arbitrary Poses").  One block
// per query walks the waypoints of each candidate solution in turn.
constexpr int kTrackMaxPoints = 1024;
struct TrackArgs {
    JointView joints[kMaxDof];   // the real arm (full limits)
    JointView vjoints[kMaxDof];  // mode 1: the virtual arm
    GridView g;
    int n, na, bx, by, bz, ia0, ie0;
    int len[kMaxDof];            // real segment lengths (reach-pose waypoints)
    int lim_lo[kMaxDof], lim_hi[kMaxDof];
    int tracked;                 // the joint that follows the waypoints (1..n)
    int delta, delta2;           // joint box per waypoint, relaxed box after a failure (steps)
    int eps2;                    // squared voxel tolerance at a waypoint
    int mode;                    // 0: reach-pose-guided, backward; 1: virtual arm, forward from start;
                                 // 2: shortcut, backward from each reach pose along guide[0..guide_k)
    int guide[kMaxDof];          // mode 2: the shortcut's joint prefix (steps)
    int guide_k, guide_s;        // mode 2: its segment and hit sample (1-based)
    int vn, vbx, vby, vbz, via0, vie0;
    int vlen[kMaxDof];
    int start[kMaxDof];          // mode 1: the start pose
    int nsol;                    // candidate solutions, tried in order
    const int32_t* sols;         // nsol * (mode 0: n, mode 1: vn) joint values in steps
    int32_t* rows;               // out: (M + 1) * n joint values in steps, in path order
    int32_t* status;             // out: [0] rows written (0: none), [1] solution used, [2] waypoints
};
hipError_t launch_track(const TrackArgs& a, hipStream_t st);
// args: device array of `count` argument blocks, one block per query
hipError_t launch_track_batch(const TrackArgs* args, int count, hipStream_t st);

struct TubeArgs {
    JointView joints[kMaxDof];
    GridView g;
    int n, na, bx, by, bz, ia0, ie0;
    int W, delta, r;
    int start[kMaxDof], goal[kMaxDof], lim_lo[kMaxDof], lim_hi[kMaxDof];
    uint64_t slab;             // (2r+1)^n cells per waypoint
};
hipError_t launch_tube_valid(const TubeArgs& a, uint8_t* valid, hipStream_t st);
// Bit-parallel search in the blocked frame layout: the plan (lds == 0: does not apply),
// then the launch (validity bits + dynamic program + backward choice in one block).
// vbits and rbits hold (W + 1) * nw words each.  With A > 1 the launch searches A
// attempts that differ only in their goal (goals: A * n values, device-readable) at once,
// one block each: attempt i's frames start (W + 1) * nw * i words into vbits and rbits,
// its rows (W + 1) * n * i values into path, its status at status[i].
struct TubeBlk {
    int q, no, b;              // inner joints, outer joints, words per block
    uint32_t Bq, nblk;         // cells per block (B^q), blocks per frame (B^no)
    uint64_t nw;               // words per frame
    size_t lds;                // dynamic LDS bytes
    int frames_lds;            // 1: the W + 1 validity and reach frames are kept in LDS
};
TubeBlk tube_blk_plan(const TubeArgs& a);
hipError_t launch_tube_bits(const TubeArgs& a, const TubeBlk& t, uint64_t* vbits, uint64_t* rbits, int32_t* path,
                            int32_t* status, hipStream_t st, int A = 1, const int32_t* goals = nullptr);
hipError_t launch_tube_solve(const TubeArgs& a, const uint8_t* valid, uint8_t* reach, uint8_t* tmp0,
                             uint8_t* tmp1, int32_t* path, int32_t* status, hipStream_t st);

}  // namespace msc
