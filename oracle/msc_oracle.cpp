// Plain CPU oracle for the staged reach search of the gap map-seeking arm solver
// (Arathorn, "Fast Robot Arm Inverse Kinematics and Path Planning Under Complex
// Static and Dynamic Obstacle Constraints", arXiv 1906.10678).
//
// TEST INFRASTRUCTURE ONLY.  This file is compiled into liborc.so, which only the
// test-suite, the smoke check and the CPU-baseline leg of the benchmark load.  It
// shares no code, header, table or helper with the GPU library: every quantity
// below is computed here from the definitions, in the order they are stated, with
// std::sort / std::unique as the only library steps.  Speed is not a goal.
//
// Discrete model (the readings are listed in the design notes of the repository):
//   * The arm is a chain of translations, each a segment length times a unit
//     direction given by azimuth and elevation in the global frame
//     (paper: Introduction, eq 1 and the vector-sum form below it; "The
//     representations of the arm and obstacles").
//   * Joint k is a yaw joint (adds to azimuth) or a pitch joint (adds to
//     elevation); joint angles are integer multiples of the step.  The state after
//     segment k is (end voxel, orientation) = (p, (ia, ie)).
//   * Segment mappings are rounded back onto the voxel grid ("conventional MSC ...
//     rounded back into the spatial representation for each step", section "The
//     representations of the arm and obstacles").
//   * Collision is tested at S equally spaced points along a segment, each rounded
//     to a voxel index and looked up in the obstacle grid (section "Testing for
//     collisions"; S = 8 in "Implementation Performance").
//   * Forward pathway from the root, backward pathway from the target, joined in
//     the middle (section "The gap in gMS"); distance pruning after eqs 5-8.
//   * One reach pose is chosen from the surviving set ("The procedure for IK
//     solution", Step 3): the first tuple in a fixed canonical order.
//
// Parity status: tables, raster, forward/backward sets, join and the canonical
// pose are pinned by closed forms, brute force and invariants in tests/.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

extern "C" {

// Arm description used by the oracle.  Angles are in steps of 360/na degrees.
struct orc_arm {
    int32_t n;           // number of joints (= segments)
    int32_t na;          // orientation bins per full turn (360 deg / step)
    int32_t S;           // collision samples per segment
    int32_t base[3];     // root voxel
    int32_t ia0, ie0;    // initial orientation (azimuth, elevation) in steps
    int32_t type[16];    // 0 = yaw (azimuth), 1 = pitch (elevation)
    int32_t len[16];     // segment length in voxels
    int32_t lo[16];      // joint lower limit in steps (inclusive)
    int32_t hi[16];      // joint upper limit in steps (inclusive)
    int32_t ref[16];     // reference angle for the canonical order, in steps
    // Approach cone of the last segment (Fig 3, the cone at the target): final
    // orientations whose direction lies within app_half_cdeg of the direction of
    // (app_az_cdeg, app_el_cdeg); app_half_cdeg < 0: no cone.
    int32_t app_az_cdeg, app_el_cdeg, app_half_cdeg;
};

}  // extern "C"

namespace {

// Direction of orientation (az, el) given in degrees: (cos el cos az, cos el sin az, sin el).
void unit_dir(double az_deg, double el_deg, double d[3]) {
    const double az = az_deg * M_PI / 180.0, el = el_deg * M_PI / 180.0;
    d[0] = std::cos(el) * std::cos(az);
    d[1] = std::cos(el) * std::sin(az);
    d[2] = std::sin(el);
}

// Is the final orientation (ia, ie) inside the arm's approach cone?  The angle to the
// axis is at most the half-angle when the dot product of the unit directions is at
// least its cosine; a band of 1e-9 keeps a boundary case inside whatever the rounding.
bool in_cone(const orc_arm& A, int ia, int ie) {
    if (A.app_half_cdeg < 0) return true;
    double a[3], d[3];
    unit_dir(A.app_az_cdeg / 100.0, A.app_el_cdeg / 100.0, a);
    const double step = 360.0 / A.na;
    unit_dir(ia * step, ie * step, d);
    const double dot = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
    return dot >= std::cos(A.app_half_cdeg / 100.0 * M_PI / 180.0) - 1e-9;
}

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Rounding of a real coordinate to a voxel index: nearest integer, exact halves
// away from zero.  A value is treated as an exact half when it lies within 1e-9
// of one, so that FP64 evaluation order cannot split a true tie (L*cos 60 deg and
// L*sin 30 deg are both exactly L/2 but differ in the last bits in FP64).
// ---------------------------------------------------------------------------
int64_t round_voxel(double v) {
    double a = std::fabs(v);
    double fl = std::floor(a);
    double frac = a - fl;
    double r;
    if (std::fabs(frac - 0.5) <= 1e-9) {
        r = fl + 1.0;
    } else {
        r = std::floor(a + 0.5);
    }
    return (int64_t)(v < 0 ? -r : r);
}

// Direction of a segment with global azimuth ia and elevation ie (in steps):
// (cos el cos az, cos el sin az, sin el), x east, y north, z up.
void direction(int na, int ia, int ie, double d[3]) {
    double az = 2.0 * kPi * (double)ia / (double)na;
    double el = 2.0 * kPi * (double)ie / (double)na;
    d[0] = std::cos(el) * std::cos(az);
    d[1] = std::cos(el) * std::sin(az);
    d[2] = std::sin(el);
}

// Tables of one segment: off[o] = round(L * d(o)); sweep[o][s] = round((s*L/S) * d(o))
// for s = 1..S.  o = ia * na + ie.
struct SegTable {
    std::vector<int32_t> off;    // na*na*3
    std::vector<int32_t> sweep;  // na*na*S*3
};

SegTable make_table(int na, int S, int L) {
    SegTable t;
    t.off.assign((size_t)na * na * 3, 0);
    t.sweep.assign((size_t)na * na * S * 3, 0);
    for (int ia = 0; ia < na; ++ia) {
        for (int ie = 0; ie < na; ++ie) {
            double d[3];
            direction(na, ia, ie, d);
            size_t o = (size_t)ia * na + ie;
            for (int c = 0; c < 3; ++c) t.off[o * 3 + c] = (int32_t)round_voxel((double)L * d[c]);
            for (int s = 1; s <= S; ++s) {
                double frac_len = (double)s * (double)L / (double)S;
                for (int c = 0; c < 3; ++c)
                    t.sweep[(o * S + (s - 1)) * 3 + c] = (int32_t)round_voxel(frac_len * d[c]);
            }
        }
    }
    return t;
}

// ---------------------------------------------------------------------------
// Obstacle grid: one byte per voxel, index (z*N + y)*N + x, 1 = blocked.
// A voxel is blocked when it lies within Euclidean distance r of a box or within
// distance R + r of a sphere centre (dilation of the obstacles for arm thickness,
// section "The representations of the arm and obstacles" and Fig 4).
// ---------------------------------------------------------------------------
struct Grid {
    int N;
    const uint8_t* occ;
    bool free_voxel(int64_t x, int64_t y, int64_t z) const {
        if (x < 0 || y < 0 || z < 0 || x >= N || y >= N || z >= N) return false;
        return occ[((size_t)z * N + (size_t)y) * N + (size_t)x] == 0;
    }
};

int64_t sq(int64_t v) { return v * v; }

// ---------------------------------------------------------------------------
// States are packed into one sorted 64-bit key: voxel index (z*N+y)*N+x in the
// high bits, then azimuth index, then elevation index (8 bits each).
// ---------------------------------------------------------------------------
uint64_t make_key(int N, int64_t x, int64_t y, int64_t z, int ia, int ie) {
    uint64_t v = ((uint64_t)z * N + (uint64_t)y) * N + (uint64_t)x;
    return (v << 16) | ((uint64_t)ia << 8) | (uint64_t)ie;
}
void split_key(int N, uint64_t key, int64_t p[3], int* ia, int* ie) {
    *ie = (int)(key & 0xff);
    *ia = (int)((key >> 8) & 0xff);
    uint64_t v = key >> 16;
    p[0] = (int64_t)(v % N);
    p[1] = (int64_t)((v / N) % N);
    p[2] = (int64_t)(v / ((uint64_t)N * N));
}

bool contains(const std::vector<uint64_t>& sorted, uint64_t key) {
    return std::binary_search(sorted.begin(), sorted.end(), key);
}

void sort_unique(std::vector<uint64_t>& v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
}

int wrap(int v, int na) {
    int r = v % na;
    return r < 0 ? r + na : r;
}

// Orientation after joint k moves by a steps from (ia, ie).
void turn(const orc_arm& arm, int k, int ia, int ie, int a, int* ia2, int* ie2) {
    if (arm.type[k] == 0) {
        *ia2 = wrap(ia + a, arm.na);
        *ie2 = ie;
    } else {
        *ia2 = ia;
        *ie2 = wrap(ie + a, arm.na);
    }
}

// A segment k laid from p along orientation o is clear when every one of its S
// sample points is inside the grid and not blocked (section "Testing for
// collisions").  The start point is the previous joint, tested by the previous
// segment (or the free base).
bool segment_clear(const Grid& g, const SegTable& t, int S, int na, const int64_t p[3],
                   int ia, int ie) {
    size_t o = (size_t)ia * na + ie;
    for (int s = 0; s < S; ++s) {
        const int32_t* w = &t.sweep[(o * S + s) * 3];
        if (!g.free_voxel(p[0] + w[0], p[1] + w[1], p[2] + w[2])) return false;
    }
    return true;
}

// ceil(sqrt(v)) for v >= 0, in integers.
int64_t isqrt_ceil(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r < v) ++r;
    while (r > 0 && (r - 1) * (r - 1) >= v) --r;
    return r;
}

struct Problem {
    orc_arm arm;
    Grid grid;
    int64_t target[3];
    int prune;                       // 1 = apply the distance pruning, 0 = off
    std::vector<SegTable> tables;    // per joint
    std::vector<int64_t> reach;      // per joint: ceil(max_o |off_k[o]|)
    std::vector<std::vector<uint8_t>> orient;  // O_k: orientations reachable after k joints
};

void prepare(Problem& P) {
    const orc_arm& A = P.arm;
    P.tables.clear();
    P.reach.clear();
    for (int k = 0; k < A.n; ++k) {
        P.tables.push_back(make_table(A.na, A.S, A.len[k]));
        int64_t m2 = 0;
        const std::vector<int32_t>& off = P.tables.back().off;
        for (size_t o = 0; o < (size_t)A.na * A.na; ++o)
            m2 = std::max(m2, sq(off[o * 3]) + sq(off[o * 3 + 1]) + sq(off[o * 3 + 2]));
        P.reach.push_back(isqrt_ceil(m2));
    }
    // O_0 = {o0}; O_k = {o turned by a : o in O_{k-1}, a in [lo_k, hi_k]}.
    P.orient.assign(A.n + 1, std::vector<uint8_t>((size_t)A.na * A.na, 0));
    P.orient[0][(size_t)wrap(A.ia0, A.na) * A.na + wrap(A.ie0, A.na)] = 1;
    for (int k = 0; k < A.n; ++k) {
        for (int ia = 0; ia < A.na; ++ia)
            for (int ie = 0; ie < A.na; ++ie) {
                if (!P.orient[k][(size_t)ia * A.na + ie]) continue;
                for (int a = A.lo[k]; a <= A.hi[k]; ++a) {
                    int ia2, ie2;
                    turn(A, k, ia, ie, a, &ia2, &ie2);
                    P.orient[k + 1][(size_t)ia2 * A.na + ie2] = 1;
                }
            }
    }
}

// Forward pruning radius after k segments (k = 1..n): the remaining segments
// k+1..n can cover at most the sum of their longest offsets (eqs 5-6).
int64_t fwd_radius(const Problem& P, int k) {
    int64_t r = 0;
    for (int j = k; j < P.arm.n; ++j) r += P.reach[j];
    return r;
}
// Backward pruning radius after k segments: the first k segments reach at most
// the sum of their longest offsets from the base (eqs 7-8).
int64_t bwd_radius(const Problem& P, int k) {
    int64_t r = 0;
    for (int j = 0; j < k; ++j) r += P.reach[j];
    return r;
}

// Forward stage k (1-based): all valid successors of the states in cur.
std::vector<uint64_t> forward_stage(const Problem& P, const std::vector<uint64_t>& cur, int k) {
    const orc_arm& A = P.arm;
    const SegTable& T = P.tables[k - 1];
    const int N = P.grid.N;
    const int64_t R = fwd_radius(P, k);
    std::vector<uint64_t> out;
    std::vector<uint64_t> chunk;
    const size_t kChunk = 1u << 22;
    for (size_t i = 0; i < cur.size(); ++i) {
        int64_t p[3];
        int ia, ie;
        split_key(N, cur[i], p, &ia, &ie);
        for (int a = A.lo[k - 1]; a <= A.hi[k - 1]; ++a) {
            int ia2, ie2;
            turn(A, k - 1, ia, ie, a, &ia2, &ie2);
            const int32_t* d = &T.off[((size_t)ia2 * A.na + ie2) * 3];
            int64_t q[3] = {p[0] + d[0], p[1] + d[1], p[2] + d[2]};
            if (P.prune) {
                int64_t d2 = sq(q[0] - P.target[0]) + sq(q[1] - P.target[1]) + sq(q[2] - P.target[2]);
                if (d2 > R * R) continue;
            }
            if (!segment_clear(P.grid, T, A.S, A.na, p, ia2, ie2)) continue;
            chunk.push_back(make_key(N, q[0], q[1], q[2], ia2, ie2));
        }
        if (chunk.size() >= kChunk || i + 1 == cur.size()) {
            sort_unique(chunk);
            std::vector<uint64_t> merged;
            merged.reserve(out.size() + chunk.size());
            std::merge(out.begin(), out.end(), chunk.begin(), chunk.end(), std::back_inserter(merged));
            merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
            out.swap(merged);
            chunk.clear();
        }
    }
    return out;
}

// Backward stage k (1-based): from the states after segment k, the states after
// segment k-1 from which one move of joint k with a clear segment k leads into cur.
std::vector<uint64_t> backward_stage(const Problem& P, const std::vector<uint64_t>& cur, int k) {
    const orc_arm& A = P.arm;
    const SegTable& T = P.tables[k - 1];
    const int N = P.grid.N;
    const int64_t R = bwd_radius(P, k - 1);
    const std::vector<uint8_t>& Oprev = P.orient[k - 1];
    std::vector<uint64_t> out;
    std::vector<uint64_t> chunk;
    const size_t kChunk = 1u << 22;
    for (size_t i = 0; i < cur.size(); ++i) {
        int64_t q[3];
        int ia2, ie2;
        split_key(N, cur[i], q, &ia2, &ie2);
        const int32_t* d = &T.off[((size_t)ia2 * A.na + ie2) * 3];
        int64_t p[3] = {q[0] - d[0], q[1] - d[1], q[2] - d[2]};
        bool keep_pos = P.grid.free_voxel(p[0], p[1], p[2]);
        if (keep_pos && P.prune) {
            int64_t d2 = sq(p[0] - P.arm.base[0]) + sq(p[1] - P.arm.base[1]) + sq(p[2] - P.arm.base[2]);
            if (d2 > R * R) keep_pos = false;
        }
        if (keep_pos && segment_clear(P.grid, T, A.S, A.na, p, ia2, ie2)) {
            for (int a = A.lo[k - 1]; a <= A.hi[k - 1]; ++a) {
                int ia, ie;
                turn(A, k - 1, ia2, ie2, -a, &ia, &ie);
                if (P.prune && !Oprev[(size_t)ia * A.na + ie]) continue;
                chunk.push_back(make_key(N, p[0], p[1], p[2], ia, ie));
            }
        }
        if (chunk.size() >= kChunk || i + 1 == cur.size()) {
            sort_unique(chunk);
            std::vector<uint64_t> merged;
            merged.reserve(out.size() + chunk.size());
            std::merge(out.begin(), out.end(), chunk.begin(), chunk.end(), std::back_inserter(merged));
            merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
            out.swap(merged);
            chunk.clear();
        }
    }
    return out;
}

// Canonical order of joint k's values: by distance to the reference angle, then by
// value.
std::vector<int> joint_order(const orc_arm& A, int k) {
    std::vector<int> v;
    for (int a = A.lo[k]; a <= A.hi[k]; ++a) v.push_back(a);
    int ref = A.ref[k];
    std::stable_sort(v.begin(), v.end(), [ref](int x, int y) {
        int dx = std::abs(x - ref), dy = std::abs(y - ref);
        if (dx != dy) return dx < dy;
        return x < y;
    });
    return v;
}

struct Result {
    int status = 0;                 // 0 = solution found, 1 = no reach
    int m = 0;                      // split point actually used
    std::vector<std::vector<uint64_t>> F;  // F_0..F_m
    std::vector<std::vector<uint64_t>> B;  // B_0..B_n (only m..n filled)
    std::vector<uint64_t> C;               // C_m
    std::vector<std::vector<uint64_t>> D;  // D_0..D_m
    std::vector<int32_t> sols;             // nsol * n joint values (steps)
    int nsol = 0;
};

// Depth-first enumeration of solutions in the canonical order (Step 3: one
// survivor is chosen, and another may be taken if its path fails).
void dfs(const Problem& P, Result& R, const std::vector<std::vector<int>>& order, int k,
         uint64_t state, std::vector<int32_t>& prefix, int want) {
    const orc_arm& A = P.arm;
    const int N = P.grid.N;
    if (R.nsol >= want) return;
    if (k == A.n) {
        R.sols.insert(R.sols.end(), prefix.begin(), prefix.end());
        R.nsol++;
        return;
    }
    int64_t p[3];
    int ia, ie;
    split_key(N, state, p, &ia, &ie);
    const SegTable& T = P.tables[k];
    for (int a : order[k]) {
        int ia2, ie2;
        turn(A, k, ia, ie, a, &ia2, &ie2);
        const int32_t* d = &T.off[((size_t)ia2 * A.na + ie2) * 3];
        int64_t q[3] = {p[0] + d[0], p[1] + d[1], p[2] + d[2]};
        if (!P.grid.free_voxel(q[0], q[1], q[2])) continue;
        uint64_t nk = make_key(N, q[0], q[1], q[2], ia2, ie2);
        // After joint k+1 (1-based) the state must extend to a full solution:
        // it lies in D_{k+1} on the forward side, in B_{k+1} on the backward side.
        bool ok = (k + 1 <= R.m) ? contains(R.D[k + 1], nk) : contains(R.B[k + 1], nk);
        if (!ok) continue;
        if (!segment_clear(P.grid, T, A.S, A.na, p, ia2, ie2)) continue;
        prefix.push_back(a);
        dfs(P, R, order, k + 1, nk, prefix, want);
        prefix.pop_back();
        if (R.nsol >= want) return;
    }
}

void solve(const Problem& P, int m, int want, Result& R) {
    const orc_arm& A = P.arm;
    const int N = P.grid.N;
    const int n = A.n;
    R = Result();
    R.m = m;
    R.F.assign(m + 1, {});
    R.B.assign(n + 1, {});
    R.D.assign(m + 1, {});
    const int64_t* t = P.target;
    int64_t base[3] = {A.base[0], A.base[1], A.base[2]};
    // The base and the target must be free voxels inside the grid.
    if (!P.grid.free_voxel(base[0], base[1], base[2]) ||
        !P.grid.free_voxel(t[0], t[1], t[2])) {
        R.status = 1;
        return;
    }
    // Forward pathway from the root (Steps 1 and 2A).
    R.F[0].push_back(make_key(N, base[0], base[1], base[2], wrap(A.ia0, A.na), wrap(A.ie0, A.na)));
    for (int k = 1; k <= m; ++k) R.F[k] = forward_stage(P, R.F[k - 1], k);
    // Backward pathway from the target: every orientation that the chain can have
    // at its last segment ends on the target.
    for (int ia = 0; ia < A.na; ++ia)
        for (int ie = 0; ie < A.na; ++ie)
            if ((!P.prune || P.orient[n][(size_t)ia * A.na + ie]) && in_cone(A, ia, ie))
                R.B[n].push_back(make_key(N, t[0], t[1], t[2], ia, ie));
    sort_unique(R.B[n]);
    for (int k = n; k > m; --k) R.B[k - 1] = backward_stage(P, R.B[k], k);
    // Join: the states reached from both ends (the surviving solution set).
    std::set_intersection(R.F[m].begin(), R.F[m].end(), R.B[m].begin(), R.B[m].end(),
                          std::back_inserter(R.C));
    if (R.C.empty()) {
        R.status = 1;
        return;
    }
    // D_m = C_m; D_{k-1} = states of F_{k-1} with a valid move into D_k.
    R.D[m] = R.C;
    for (int k = m; k >= 1; --k) {
        const SegTable& T = P.tables[k - 1];
        for (uint64_t s : R.F[k - 1]) {
            int64_t p[3];
            int ia, ie;
            split_key(N, s, p, &ia, &ie);
            bool any = false;
            for (int a = A.lo[k - 1]; a <= A.hi[k - 1] && !any; ++a) {
                int ia2, ie2;
                turn(A, k - 1, ia, ie, a, &ia2, &ie2);
                const int32_t* d = &T.off[((size_t)ia2 * A.na + ie2) * 3];
                int64_t q[3] = {p[0] + d[0], p[1] + d[1], p[2] + d[2]};
                if (!P.grid.free_voxel(q[0], q[1], q[2])) continue;
                if (!contains(R.D[k], make_key(N, q[0], q[1], q[2], ia2, ie2))) continue;
                if (!segment_clear(P.grid, T, A.S, A.na, p, ia2, ie2)) continue;
                any = true;
            }
            if (any) R.D[k - 1].push_back(s);
        }
    }
    std::vector<std::vector<int>> order;
    for (int k = 0; k < n; ++k) order.push_back(joint_order(A, k));
    std::vector<int32_t> prefix;
    dfs(P, R, order, 0, R.F[0][0], prefix, want);
    R.status = R.nsol > 0 ? 0 : 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points (loaded through ctypes by the tests).
// ---------------------------------------------------------------------------
extern "C" {

// off: na*na*3, sweep: na*na*S*3 (int32).  Entry o = ia*na + ie.
int orc_tables(int32_t na, int32_t S, int32_t L, int32_t* off, int32_t* sweep) {
    if (na <= 0 || S <= 0 || L < 0) return -1;
    SegTable t = make_table(na, S, L);
    std::memcpy(off, t.off.data(), t.off.size() * sizeof(int32_t));
    std::memcpy(sweep, t.sweep.data(), t.sweep.size() * sizeof(int32_t));
    return 0;
}

// boxes: nbox * 6 (lo xyz, extent xyz); spheres: nsph * 4 (centre xyz, radius).
// occ: N*N*N bytes, index (z*N + y)*N + x, written 1 where blocked.
int orc_raster(int32_t N, int32_t r, const int32_t* boxes, int32_t nbox, const int32_t* spheres,
               int32_t nsph, uint8_t* occ) {
    if (N <= 0 || r < 0) return -1;
    for (int64_t z = 0; z < N; ++z)
        for (int64_t y = 0; y < N; ++y)
            for (int64_t x = 0; x < N; ++x) {
                int64_t v[3] = {x, y, z};
                bool blocked = false;
                for (int i = 0; i < nbox && !blocked; ++i) {
                    const int32_t* bx = &boxes[i * 6];
                    int64_t d2 = 0;
                    for (int c = 0; c < 3; ++c) {
                        int64_t lo = bx[c], hi = (int64_t)bx[c] + bx[3 + c] - 1;
                        int64_t e = 0;
                        if (v[c] < lo) e = lo - v[c];
                        if (v[c] > hi) e = v[c] - hi;
                        d2 += e * e;
                    }
                    if (d2 <= (int64_t)r * r) blocked = true;
                }
                for (int i = 0; i < nsph && !blocked; ++i) {
                    const int32_t* s = &spheres[i * 4];
                    int64_t d2 = sq(x - s[0]) + sq(y - s[1]) + sq(z - s[2]);
                    int64_t rr = (int64_t)s[3] + r;
                    if (d2 <= rr * rr) blocked = true;
                }
                occ[((size_t)z * N + (size_t)y) * N + (size_t)x] = blocked ? 1 : 0;
            }
    return 0;
}

// Forward kinematics replay of one pose q (n joint values in steps): returns 1 if
// every segment is clear (and the base is free), 0 otherwise; end receives the
// end voxel, joints receives the n+1 joint voxels (base first) if not null.
int orc_pose(const orc_arm* arm, int32_t N, const uint8_t* occ, const int32_t* q, int64_t* end,
             int64_t* joints) {
    const orc_arm& A = *arm;
    Grid g{N, occ};
    int64_t p[3] = {A.base[0], A.base[1], A.base[2]};
    int ia = wrap(A.ia0, A.na), ie = wrap(A.ie0, A.na);
    bool ok = g.free_voxel(p[0], p[1], p[2]);
    if (joints) for (int c = 0; c < 3; ++c) joints[c] = p[c];
    for (int k = 0; k < A.n; ++k) {
        SegTable T = make_table(A.na, A.S, A.len[k]);
        int ia2, ie2;
        turn(A, k, ia, ie, q[k], &ia2, &ie2);
        if (!segment_clear(g, T, A.S, A.na, p, ia2, ie2)) ok = false;
        const int32_t* d = &T.off[((size_t)ia2 * A.na + ie2) * 3];
        for (int c = 0; c < 3; ++c) p[c] += d[c];
        ia = ia2;
        ie = ie2;
        if (joints) for (int c = 0; c < 3; ++c) joints[(k + 1) * 3 + c] = p[c];
    }
    if (end) for (int c = 0; c < 3; ++c) end[c] = p[c];
    return ok ? 1 : 0;
}

// Batched pose replay: q is count*n; valid receives count bytes; ends count*3.
int orc_pose_batch(const orc_arm* arm, int32_t N, const uint8_t* occ, const int32_t* q,
                   int64_t count, uint8_t* valid, int64_t* ends) {
    const orc_arm& A = *arm;
    Grid g{N, occ};
    std::vector<SegTable> tabs;
    for (int k = 0; k < A.n; ++k) tabs.push_back(make_table(A.na, A.S, A.len[k]));
    for (int64_t i = 0; i < count; ++i) {
        int64_t p[3] = {A.base[0], A.base[1], A.base[2]};
        int ia = wrap(A.ia0, A.na), ie = wrap(A.ie0, A.na);
        bool ok = g.free_voxel(p[0], p[1], p[2]);
        for (int k = 0; k < A.n; ++k) {
            int ia2, ie2;
            turn(A, k, ia, ie, q[i * A.n + k], &ia2, &ie2);
            if (ok && !segment_clear(g, tabs[k], A.S, A.na, p, ia2, ie2)) ok = false;
            const int32_t* d = &tabs[k].off[((size_t)ia2 * A.na + ie2) * 3];
            for (int c = 0; c < 3; ++c) p[c] += d[c];
            ia = ia2;
            ie = ie2;
        }
        valid[i] = ok ? 1 : 0;
        if (ends) for (int c = 0; c < 3; ++c) ends[i * 3 + c] = p[c];
    }
    return 0;
}

// Continuous FP64 forward kinematics (no rounding): the end point of the chain.
int orc_pose_continuous(const orc_arm* arm, const int32_t* q, double* end) {
    const orc_arm& A = *arm;
    double p[3] = {(double)A.base[0], (double)A.base[1], (double)A.base[2]};
    int ia = wrap(A.ia0, A.na), ie = wrap(A.ie0, A.na);
    for (int k = 0; k < A.n; ++k) {
        int ia2, ie2;
        turn(A, k, ia, ie, q[k], &ia2, &ie2);
        double d[3];
        direction(A.na, ia2, ie2, d);
        for (int c = 0; c < 3; ++c) p[c] += (double)A.len[k] * d[c];
        ia = ia2;
        ie = ie2;
    }
    for (int c = 0; c < 3; ++c) end[c] = p[c];
    return 0;
}

// Orientation reachability O_k (k = 0..n), out: (n+1) * na * na bytes.
int orc_orientations(const orc_arm* arm, uint8_t* out) {
    Problem P;
    P.arm = *arm;
    P.grid = Grid{1, nullptr};
    prepare(P);
    size_t sz = (size_t)arm->na * arm->na;
    for (int k = 0; k <= arm->n; ++k) std::memcpy(out + k * sz, P.orient[k].data(), sz);
    return 0;
}

// Pruning radii: reach[k] = ceil(max_o |off_k[o]|) for k = 0..n-1.
int orc_reach_radii(const orc_arm* arm, int64_t* reach) {
    Problem P;
    P.arm = *arm;
    P.grid = Grid{1, nullptr};
    prepare(P);
    for (int k = 0; k < arm->n; ++k) reach[k] = P.reach[k];
    return 0;
}

// Staged reach search.  Returns a handle to the result (free with orc_free).
// m: split point (0..n).  want: how many solutions to enumerate in canonical order.
void* orc_solve(const orc_arm* arm, int32_t N, const uint8_t* occ, const int32_t* target,
                int32_t m, int32_t want, int32_t prune) {
    if (m < 0 || m > arm->n || arm->n < 1 || arm->n > 16) return nullptr;
    Problem P;
    P.arm = *arm;
    P.grid = Grid{N, occ};
    for (int c = 0; c < 3; ++c) P.target[c] = target[c];
    P.prune = prune;
    prepare(P);
    Result* R = new Result();
    solve(P, m, want, *R);
    return R;
}

int orc_status(void* h) { return ((Result*)h)->status; }
int orc_split(void* h) { return ((Result*)h)->m; }
int orc_nsol(void* h) { return ((Result*)h)->nsol; }
void orc_sols(void* h, int32_t* out) {
    Result* R = (Result*)h;
    std::memcpy(out, R->sols.data(), R->sols.size() * sizeof(int32_t));
}
// which: 0 = F, 1 = B, 2 = C, 3 = D.  Returns the size; copies if out != null.
int64_t orc_set(void* h, int32_t which, int32_t stage, uint64_t* out) {
    Result* R = (Result*)h;
    const std::vector<uint64_t>* v = nullptr;
    if (which == 0 && stage >= 0 && stage < (int)R->F.size()) v = &R->F[stage];
    if (which == 1 && stage >= 0 && stage < (int)R->B.size()) v = &R->B[stage];
    if (which == 2) v = &R->C;
    if (which == 3 && stage >= 0 && stage < (int)R->D.size()) v = &R->D[stage];
    if (!v) return -1;
    if (out) std::memcpy(out, v->data(), v->size() * sizeof(uint64_t));
    return (int64_t)v->size();
}
void orc_free(void* h) { delete (Result*)h; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Brute force, for tiny arms only: no staging and no de-duplication.
// ---------------------------------------------------------------------------
namespace {

struct Brute {
    const Problem* P;
    std::vector<std::vector<uint64_t>> F;  // per stage, unsorted, then sorted
    std::vector<std::vector<uint64_t>> B;
};

// Every prefix of joint values from the base, cut where a segment collides (and,
// with pruning on, where the prefix end is out of the forward radius).
void brute_forward(Brute& Z, int k, const int64_t p[3], int ia, int ie, int kmax) {
    const Problem& P = *Z.P;
    const orc_arm& A = P.arm;
    Z.F[k].push_back(make_key(P.grid.N, p[0], p[1], p[2], ia, ie));
    if (k == kmax) return;
    for (int a = A.lo[k]; a <= A.hi[k]; ++a) {
        int ia2, ie2;
        turn(A, k, ia, ie, a, &ia2, &ie2);
        if (!segment_clear(P.grid, P.tables[k], A.S, A.na, p, ia2, ie2)) continue;
        const int32_t* d = &P.tables[k].off[((size_t)ia2 * A.na + ie2) * 3];
        int64_t q[3] = {p[0] + d[0], p[1] + d[1], p[2] + d[2]};
        if (P.prune) {
            int64_t R = fwd_radius(P, k + 1);
            if (sq(q[0] - P.target[0]) + sq(q[1] - P.target[1]) + sq(q[2] - P.target[2]) > R * R) continue;
        }
        brute_forward(Z, k + 1, q, ia2, ie2, kmax);
    }
}

// Every suffix of joint values ending at the target, walked back from the target.
void brute_backward(Brute& Z, int k, const int64_t q[3], int ia2, int ie2, int kmin) {
    const Problem& P = *Z.P;
    const orc_arm& A = P.arm;
    Z.B[k].push_back(make_key(P.grid.N, q[0], q[1], q[2], ia2, ie2));
    if (k == kmin) return;
    const int32_t* d = &P.tables[k - 1].off[((size_t)ia2 * A.na + ie2) * 3];
    int64_t p[3] = {q[0] - d[0], q[1] - d[1], q[2] - d[2]};
    if (!P.grid.free_voxel(p[0], p[1], p[2])) return;
    if (!segment_clear(P.grid, P.tables[k - 1], A.S, A.na, p, ia2, ie2)) return;
    if (P.prune) {
        int64_t R = bwd_radius(P, k - 1);
        if (sq(p[0] - A.base[0]) + sq(p[1] - A.base[1]) + sq(p[2] - A.base[2]) > R * R) return;
    }
    for (int a = A.lo[k - 1]; a <= A.hi[k - 1]; ++a) {
        int ia, ie;
        turn(A, k - 1, ia2, ie2, -a, &ia, &ie);
        if (P.prune && !P.orient[k - 1][(size_t)ia * A.na + ie]) continue;
        brute_backward(Z, k - 1, p, ia, ie, kmin);
    }
}

Brute* g_brute = nullptr;

}  // namespace

extern "C" {

// Per-stage sets by exhaustive prefix / suffix enumeration: forward sets for
// stages 0..kf, backward sets for stages kb..n.  Read them with orc_brute_set.
int orc_brute_sets(const orc_arm* arm, int32_t N, const uint8_t* occ, const int32_t* target,
                   int32_t kf, int32_t kb, int32_t prune) {
    static Problem P;
    P = Problem();
    P.arm = *arm;
    P.grid = Grid{N, occ};
    for (int c = 0; c < 3; ++c) P.target[c] = target[c];
    P.prune = prune;
    prepare(P);
    delete g_brute;
    g_brute = new Brute();
    g_brute->P = &P;
    g_brute->F.assign(arm->n + 1, {});
    g_brute->B.assign(arm->n + 1, {});
    const orc_arm& A = P.arm;
    int64_t base[3] = {A.base[0], A.base[1], A.base[2]};
    if (!P.grid.free_voxel(base[0], base[1], base[2]) ||
        !P.grid.free_voxel(target[0], target[1], target[2]))
        return 1;
    brute_forward(*g_brute, 0, base, wrap(A.ia0, A.na), wrap(A.ie0, A.na), kf);
    int64_t t[3] = {target[0], target[1], target[2]};
    for (int ia = 0; ia < A.na; ++ia)
        for (int ie = 0; ie < A.na; ++ie)
            if ((!prune || P.orient[A.n][(size_t)ia * A.na + ie]) && in_cone(A, ia, ie))
                brute_backward(*g_brute, A.n, t, ia, ie, kb);
    for (auto& v : g_brute->F) sort_unique(v);
    for (auto& v : g_brute->B) sort_unique(v);
    return 0;
}

int64_t orc_brute_set(int32_t which, int32_t stage, uint64_t* out) {
    if (!g_brute) return -1;
    std::vector<uint64_t>& v = which == 0 ? g_brute->F[stage] : g_brute->B[stage];
    if (out) std::memcpy(out, v.data(), v.size() * sizeof(uint64_t));
    return (int64_t)v.size();
}

// All joint tuples whose replay is clear and ends on the target, in the canonical
// order (distance of each joint to its reference, then value, joint 1 first).
// Writes up to cap tuples into out and returns the total count.
int64_t orc_brute_solutions(const orc_arm* arm, int32_t N, const uint8_t* occ,
                            const int32_t* target, int64_t cap, int32_t* out) {
    const orc_arm& A = *arm;
    const int n = A.n;
    std::vector<std::vector<int>> order;
    for (int k = 0; k < n; ++k) order.push_back(joint_order(A, k));
    // Odometer over the canonical orders, so that the enumeration itself runs in
    // the canonical (lexicographic) order.  Tuples are replayed in chunks.
    std::vector<int> idx(n, 0);
    const int64_t kChunk = 1 << 16;
    std::vector<int32_t> tuples;
    std::vector<uint8_t> ok(kChunk);
    std::vector<int64_t> ends(kChunk * 3);
    int64_t count = 0;
    bool done = false;
    while (!done) {
        tuples.clear();
        while ((int64_t)tuples.size() < kChunk * n && !done) {
            for (int k = 0; k < n; ++k) tuples.push_back(order[k][idx[k]]);
            int k = n - 1;
            while (k >= 0) {
                if (++idx[k] < (int)order[k].size()) break;
                idx[k] = 0;
                --k;
            }
            if (k < 0) done = true;
        }
        int64_t cnt = (int64_t)tuples.size() / n;
        orc_pose_batch(arm, N, occ, tuples.data(), cnt, ok.data(), ends.data());
        for (int64_t i = 0; i < cnt; ++i) {
            if (!ok[i] || ends[i * 3] != target[0] || ends[i * 3 + 1] != target[1] ||
                ends[i * 3 + 2] != target[2])
                continue;
            if (count < cap) std::memcpy(out + count * n, &tuples[i * n], n * sizeof(int32_t));
            ++count;
        }
    }
    return count;
}

}  // extern "C"
