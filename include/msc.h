/*
 * msc.h - C ABI of the MI355X staged reach / path solver.
 *
 * The solver implements the data-parallel search of the gap map-seeking arm method
 * (Arathorn, arXiv 1906.10678) on a voxel grid:
 *   - an arm is a chain of segments whose directions are azimuth / elevation in the
 *     global frame (Introduction, eq 1 and its vector-sum form);
 *   - obstacles are a voxel grid, dilated for arm thickness (section "The
 *     representations of the arm and obstacles", Fig 4);
 *   - a segment collides if any of its S equally spaced sample points falls in a
 *     blocked voxel (section "Testing for collisions");
 *   - the reachable (joint voxel, orientation) states are expanded stage by stage
 *     from the root (forward pathway) and from the target (backward pathway) and
 *     intersected (section "The gap in gMS", eqs 5-8 for the distance pruning;
 *     "The procedure for IK solution", Steps 1-3);
 *   - one survivor is chosen as the reach pose, and a smooth waypoint path to it
 *     is searched backward from the reach pose (sections "Smooth sequence
 *     computation" and "Filtering for smoothness").
 *
 * Units and conventions
 *   - Voxel coordinates are integers 0..n-1 per axis; x east, y north, z up.
 *   - Angles are int32 centidegrees.  step_cdeg must divide 36000 and the number of
 *     orientation bins 36000/step_cdeg must be <= 256.  Joint limits, the initial
 *     orientation and start poses must be multiples of step_cdeg.
 *   - A yaw joint adds its angle to the segment azimuth, a pitch joint to the
 *     elevation; segment k points along (cos el cos az, cos el sin az, sin el).
 *   - Segment mappings and sample points are rounded to the nearest voxel, exact
 *     halves away from zero.
 *
 * Ownership
 *   - Every input pointer is read during the call and not retained.
 *   - Handles are created by *_create and released by *_destroy.
 *   - Output pointers are caller-allocated host buffers of the documented size.
 *   - Device memory is caller-provided: msc_ctx_create receives a device workspace
 *     and msc_scene_create a device buffer for the occupancy grid.  The library
 *     sub-allocates from them and calls no device allocator of its own.
 *
 * Errors
 *   - 0 = success; positive = a valid "no answer" result; negative = error.
 *   - On a negative status nothing is written to the outputs and msc_last_error()
 *     returns a message.  No C++ exception crosses this interface.
 *
 * Synchronisation
 *   - All device work is enqueued on the stream given to msc_ctx_create.  Every call
 *     below returns after its results are on the host.
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef MSC_H
#define MSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSC_MAX_DOF 16

typedef enum {
    MSC_OK = 0,          /* solution written */
    MSC_NO_REACH = 1,    /* no pose reaches the target (empty surviving set) */
    MSC_NO_PATH = 2,     /* reach poses exist, but no tube path within the retries */
    MSC_E_ARG = -1,      /* invalid argument */
    MSC_E_NOMEM = -2,    /* workspace or grid buffer too small */
    MSC_E_HIP = -3,      /* HIP runtime error */
    MSC_E_CAPACITY = -4, /* an internal table overflowed its planned capacity */
    MSC_E_STATE = -5     /* call not valid in the current state */
} msc_status;

typedef enum { MSC_YAW = 0, MSC_PITCH = 1 } msc_joint;

/* Arm chain.  Joint k (0-based) turns by an angle in [lo_cdeg[k], hi_cdeg[k]] and is
 * followed by segment k of len_vox[k] voxels (>= 0).  dof in 1..MSC_MAX_DOF;
 * samples (collision points per segment, S) >= 1; base = root voxel; the chain starts
 * with azimuth az0_cdeg and elevation el0_cdeg (9000 = straight up). */
typedef struct {
    int32_t dof, step_cdeg, samples;
    int32_t base[3];
    int32_t az0_cdeg, el0_cdeg;
    int32_t type[MSC_MAX_DOF];
    int32_t len_vox[MSC_MAX_DOF];
    int32_t lo_cdeg[MSC_MAX_DOF];
    int32_t hi_cdeg[MSC_MAX_DOF];
} msc_arm;

/* Axis-aligned box covering voxels lo .. lo+ext-1 per axis (ext >= 1). */
typedef struct { int32_t lo[3], ext[3]; } msc_box;
/* Sphere of voxels within distance r of centre c (r >= 0). */
typedef struct { int32_t c[3], r; } msc_sphere;

#define MSC_CAPTURE_SETS 1u /* keep every stage set for msc_debug_set */
#define MSC_NO_PRUNE 2u     /* disable the distance / orientation pruning (tests) */
#define MSC_PROFILE 4u      /* time every kernel launch of the call with HIP events */
#define MSC_FUSED_TRACK 8u  /* msc_batch: the waypoint tracking of every kind 2 / 3 query runs in
                               one launch after all their searches (one block per query) */
#define MSC_COUNT_SETS 16u  /* measurement: every stage set gets a member count (also the one the
                               meet probes) and, with MSC_PROFILE, each expansion's record its
                               output's non-zero words (extra kernels, outside the timed launches) */

typedef struct {
    int32_t split_m;       /* forward stages before the join: -1 = adaptive, else 0..dof */
    int32_t tube_r0;       /* first tube radius of the path search, in steps (default 1) */
    int32_t tube_r1;       /* relaxed tube radius after a failure (default 2) */
    int32_t reach_retries; /* reach poses tried by msc_path, in canonical order (default 4) */
    uint32_t flags;        /* MSC_CAPTURE_SETS | MSC_NO_PRUNE */
    /* Approach cone of the last segment (the cone at the target in Fig 3): only final
     * orientations (ia, ie) whose direction d = (cos el cos az, cos el sin az, sin el),
     * az = ia * step, el = ie * step, satisfies d . a >= cos(half) - 1e-9, where a is the
     * direction of (approach_az_cdeg, approach_el_cdeg), are offered to the backward
     * pathway.  Evaluated on the host in FP64.  approach_half_cdeg < 0 (the default)
     * disables the cone; 0..18000 is the half-angle in centidegrees. */
    int32_t approach_az_cdeg;
    int32_t approach_el_cdeg;
    int32_t approach_half_cdeg;
} msc_opts;

typedef struct msc_ctx msc_ctx;
typedef struct msc_scene msc_scene;

/* Fill *opts with the defaults {-1, 1, 2, 4, 0, 0, 0, -1} (no approach cone). */
void msc_opts_default(msc_opts* opts);

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t,
 * may be NULL for the null stream) and sub-allocates device memory from
 * [dev_workspace, dev_workspace + ws_bytes) (256-byte aligned).  The workspace must stay
 * valid until msc_ctx_destroy.  E_ARG if a pointer is NULL or ws_bytes < 64 MiB. */
msc_status msc_ctx_create(int device, void* hip_stream, void* dev_workspace, uint64_t ws_bytes,
                          msc_ctx** out);
msc_status msc_ctx_destroy(msc_ctx* ctx);

/* Device bytes needed by the occupancy grid of an n^3 scene. */
uint64_t msc_scene_bytes(int32_t n);

/* Rasterise a scene into the caller's device buffer dev_grid (msc_scene_bytes(n) bytes,
 * or msc_scene_bytes_dynamic(n, ticks) for a scene with moving obstacles):
 * a voxel is blocked when it lies within Euclidean distance dilate_r of a box or within
 * r + dilate_r of a sphere centre ("The representations of the arm and obstacles":
 * obstacles masked in a voxel array, dilated for thickness and clearance).  Voxels
 * outside the grid count as blocked.  The grid is bit-packed, 64 x-voxels per 64-bit
 * word, rows (z, y).  n in 1..1024, dilate_r >= 0. */
msc_status msc_scene_create(msc_ctx* ctx, int32_t n, int32_t dilate_r, const msc_box* boxes,
                            int32_t nbox, const msc_sphere* spheres, int32_t nsph, void* dev_grid,
                            uint64_t grid_bytes, msc_scene** out);
msc_status msc_scene_destroy(msc_scene* scene);

/* Moving obstacles ("Dynamic Obstacles": obstacles detected while the arm moves, the
 * voxel mask updated as they move).  A scene whose grid buffer holds
 * msc_scene_bytes_dynamic(n, ticks) bytes (ticks in 1..64) keeps its static grid and
 * up to `ticks` grids of recent logical ticks; returns 0 for bad arguments. */
uint64_t msc_scene_bytes_dynamic(int32_t n, int32_t ticks);

/* The scene's grid for logical tick `tick`: the static obstacles of msc_scene_create
 * plus the boxes[nbox] of this tick, dilated by the same radius, written into a grid
 * of a tick that no query is using (the oldest such; the current grid only when no other
 * is free), asynchronously on the context's stream.  The new grid becomes the scene's current grid: msc_reach / msc_path /
 * msc_pose_check / msc_debug_raster calls made afterwards see it, and so do queries
 * submitted to the server afterwards (msc_server_submit binds a query to the grid of
 * its submission tick, so its result does not depend on later ticks or on the other
 * queries in flight).  Errors: E_NOMEM if the buffer holds no grids of ticks,
 * E_CAPACITY if every grid of a tick is still in use, E_ARG for a box extent < 1.
 * Called from the thread that owns the context. */
msc_status msc_scene_set_dynamic(msc_scene* scene, const msc_box* boxes, int32_t nbox, int64_t tick);

/* Reach pose ("The procedure for IK solution", Steps 1-3).  Writes the first pose of
 * the canonical order into angles_out[dof] (centidegrees): joint tuples ordered
 * lexicographically, joint 1 first, each joint by |angle| then angle.  Returns
 * MSC_NO_REACH if no pose ends on the target with every segment clear (also when the
 * base or the target voxel is blocked).  opts may be NULL for the defaults. */
msc_status msc_reach(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm,
                     const int32_t target[3], const msc_opts* opts, int32_t* angles_out);

/* Reach pose + smooth path ("Path Planning", "Smooth sequence computation",
 * "Filtering for smoothness").  start_cdeg[dof] must be a valid pose within the limits.
 * Every joint is limited to start +- waypoints*max_delta for the reach search, whose
 * canonical order is centred on the start pose; the path is searched in a tube around
 * the straight joint-space guide from the start to the reach pose, each move changing
 * every joint by at most max_delta_cdeg, chosen backward from the reach pose (closest
 * to the guide, L1 in steps, ties by joint values); the tube radius is relaxed from
 * tube_r0 to tube_r1 after a failure, then the next reach pose is tried, up to
 * reach_retries; the path returned is that of the first attempt in this order that has
 * one (after a failed first attempt, later attempts are searched in groups, one launch
 * per radius, which changes no answer).  path_out receives (waypoints+1)*dof
 * centidegrees, row 0 = start,
 * last row = reach pose.  max_delta_cdeg must be a positive multiple of step_cdeg.
 * Returns MSC_NO_REACH or MSC_NO_PATH when no result exists. */
msc_status msc_path(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm,
                    const int32_t* start_cdeg, const int32_t target[3], int32_t waypoints,
                    int32_t max_delta_cdeg, const msc_opts* opts, int32_t* path_out);

/* Midcourse replanning ("Dynamic Obstacles": of the new paths, the one with the least
 * mean distance to the original path).  Arguments and result as msc_path, plus
 * ref_cdeg[(waypoints+1)*dof], the original path's rows to compare with (centidegrees,
 * multiples of the step; row 0 need not equal the start).  Instead of the first path
 * found, every one of the first reach_retries reach poses in the canonical order is
 * tried (tube radius tube_r0, then tube_r1) and the path with the smallest sum over the
 * waypoints of the L1 joint distance in steps to ref is returned; the earlier reach
 * pose keeps a tie.  MSC_NO_PATH if no reach pose gives a path. */
msc_status msc_replan(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm,
                      const int32_t* start_cdeg, const int32_t target[3], int32_t waypoints,
                      int32_t max_delta_cdeg, const int32_t* ref_cdeg, const msc_opts* opts,
                      int32_t* path_out);

/* Waypoint tracking of the workspace-guided paths.  At each waypoint the pose is chosen
 * among the poses whose every joint is within max_delta_cdeg of the previous pose (and
 * within the arm's limits), that are clear of obstacles (as msc_pose_check) and whose
 * joint `tracked` (the end of the first `tracked` segments) lies within squared distance
 * eps2_vox (voxels) of the waypoint: the smallest L1 joint change in steps, then the
 * smallest squared distance, then the canonical order centred on the previous pose (per
 * joint |change| then change, joint 1 first).  When there is none the box is widened to
 * relaxed_delta_cdeg for that waypoint ("Filtering for smoothness": relaxed adaptively,
 * after a failure); when that fails too, the next candidate solution is tried.
 * Defaults (msc_track_default): tracked -1 (msc_guided_path: dof - 2, msc_pose_path: dof),
 * max_delta one step, relaxed_delta two steps (-1 each), eps2_vox 9.  Requirements:
 * 0 <= max_delta <= relaxed_delta, multiples of the step; (2 relaxed/step + 1)^dof < 2^42;
 * eps2_vox in 0..1023. */
typedef struct {
    int32_t tracked;
    int32_t max_delta_cdeg;
    int32_t relaxed_delta_cdeg;
    int32_t eps2_vox;
} msc_track;
void msc_track_default(msc_track* t);

/* Reach-pose-guided path ("Path Planning", "Smooth sequence computation"): the reach
 * search of msc_reach (unwindowed, canonical order centred on 0) gives up to
 * opts->reach_retries reach poses; for each in turn, the tracked joint walks back along
 * the pose's own collision sample points, of segments tracked .. 2 (each from its end
 * to its start, segments of length 0 have none), to the end of segment 1 (the root of
 * the moving part of the arm: segment 1 rises along the initial orientation and its
 * joint only spins it), one waypoint per sample, each pose chosen from the previous one
 * as described for msc_track.  The first reach pose whose walk completes gives the path:
 * path_out receives its M + 1 rows in execution order (row 0 = the pose at the root
 * waypoint, the last row = the reach pose), M = samples * (segments of nonzero length
 * among 2..tracked), and *rows_out = M + 1.  path_out must hold
 * (samples * (tracked - 1) + 1) * dof values.  MSC_NO_REACH as msc_reach; MSC_NO_PATH when
 * no walk completes.  track may be NULL for the defaults. */
msc_status msc_guided_path(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm, const int32_t target[3],
                           const msc_track* track, const msc_opts* opts, int32_t* path_out, int32_t* rows_out);

/* Path between arbitrary poses ("Path between Arbitrary Poses"): a virtual arm
 * (virtual_arm; its base is replaced by the voxel of joint `tracked` of the start pose,
 * its step must equal the arm's) reaches for the target with the search of msc_reach;
 * for each of its first opts->reach_retries poses in turn, the real arm's tracked joint
 * follows the virtual pose's collision sample points from its root outward (segments
 * 1..V, s = 1..samples each; the last is the target), forward from the start pose, each
 * pose chosen from the previous one as described for msc_track.  path_out receives the
 * M + 1 rows (row 0 = the start pose), M = samples of the virtual arm * its segments of
 * nonzero length, and *rows_out = M + 1; it must hold (virtual samples * virtual dof + 1)
 * * dof values.  E_ARG if the start pose is not clear; MSC_NO_REACH if the virtual arm
 * cannot reach the target; MSC_NO_PATH if no walk completes. */
msc_status msc_pose_path(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm, const int32_t* start_cdeg,
                         const int32_t target[3], const msc_arm* virtual_arm, const msc_track* track,
                         const msc_opts* opts, int32_t* path_out, int32_t* rows_out);

/* Short reaches ("Short Reaches"): as the reach search tests segment hypotheses for
 * collision along their length, it also tests them for a near encounter with the target.
 * A hypothesis of segment k (k = 2..segments; segment 1 is the column the first joint only
 * spins) is a reachable state after joint k-1 and an angle of joint k; it hits the target
 * at its first sample point within squared distance rho2_vox of the target when every
 * earlier sample is free and inside the grid.  The shortcut is the hit with the least
 * path length along the arm (samples * (L_1 + ... + L_{k-1}) + s * L_k, in 1/samples
 * voxel), then the least squared distance, then the least k, realised by the first joint
 * prefix in the canonical order (reference 0).  With a hit, the end effector walks the
 * shortcut back from the target (the hit sample and the earlier samples of segment k,
 * segments k-1..2 end to start, then the end of segment 1), from each of the first
 * opts->reach_retries reach poses of msc_reach in turn, as msc_guided_path walks (the
 * track parameters; the tracked joint is the end effector); without a hit the result is
 * that of msc_guided_path.  path_out receives the rows (root waypoint pose first, reach
 * pose last) and *rows_out their number; it must hold (samples * max(segments - 1,
 * tracked - 1) + 2) * dof values.  hit_out[MSC_MAX_DOF + 3] receives k (0: no hit), the
 * hit sample s, the length, then the prefix's k joint angles (centidegrees).
 * Requirements: segments in 2..dof-1, rho2_vox in 0..65535, and ceil(sqrt(rho2_vox)) + 1
 * no more than the reach of each segment 3..segments+1 (so the pruned search keeps every
 * hit); else E_ARG.  MSC_NO_REACH / MSC_NO_PATH as msc_guided_path. */
msc_status msc_short_path(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm, const int32_t target[3],
                          int32_t rho2_vox, int32_t segments, const msc_track* track, const msc_opts* opts,
                          int32_t* path_out, int32_t* rows_out, int32_t* hit_out);

/* The paper's own search ("Discretization of the segment articulations", "The gap in
 * gMS" eqs 2-8, "The procedure for IK solution" Steps 1-3): a four-segment arm whose
 * segments 1, 2 and 4 point along vectors of a quiver, an approximately equal-area tiling
 * of the sphere, and whose segment 3 is a free vector across the gap.
 *
 * Quiver of step D = step_cdeg / 100 degrees (D divides 180 and is at least 0.2, so
 * that the quiver has fewer than 2^20 vectors; n = 360 / D): elevations
 * e_i = -90 + i D, i = 0..180/D; ring i has 1 vector at a pole, else max(min_ring,
 * round(n cos e_i)) (halves away from zero, 1e-9 band), azimuths a_ij = (j * 360) / m_i;
 * vector (cos e cos a, cos e sin a, sin e) in FP64, radians = (degrees * pi) / 180; flat
 * index = vectors of the rings below + j.
 *
 * Search (positions numerical, FP64): p1 = base + L1 r_i, p2 = p1 + L2 r_j, p3 = target -
 * L4 r_l, v3 = p3 - p2.  (i, j, l) is a solution when: r_i's elevation >= seg1_min_el;
 * |p1 - t|^2 <= (L2 + L3 + L4 + eps)^2 and |p2 - t|^2 <= (L3 + L4 + eps)^2 (eqs 5-8,
 * widened by eps); (L3 - eps)^2 <= |v3|^2 <= (L3 + eps)^2; the flexion between
 * consecutive segment directions is within max_flex_cdeg (u . v >= cos(limit) - 1e-9 |v|,
 * for v3 decided on squares); r_l inside the approach cone (r_l . a >= cos(half) - 1e-9;
 * half < 0: any); every segment clear: samples p + (s / samples) w, s = 1..samples,
 * rounded per component (halves away, 1e-9 band) in the grid and free; base and target
 * voxels free.  No operation is contracted into a fused multiply-add.
 * Outputs: *count_out = number of solutions; the first min(want, count) in (i, j, l)
 * order into sols_out[want*3] and their vectors into vec_out[want*18] (s1, s2, v3, s4,
 * then the exact s3 = v3 L3 / |v3| and s4' = (t - p2) - s3 of the 8-DOF text);
 * *nsol_out = how many were written.  MSC_NO_REACH when there is none. */
typedef struct {
    double len[4];
    int32_t base[3];
    int32_t step_cdeg;
    int32_t min_ring;
    int32_t samples;
    int32_t seg1_min_el_cdeg;
    int32_t max_flex_cdeg[3];
    int32_t approach_az_cdeg, approach_el_cdeg, approach_half_cdeg;
    double eps;
} msc_gms_arm;
/* The quiver's vectors (host only): fills min(cap, count) of them into out[cap*3] and
 * returns the count (0 for a bad step, below 20 or not dividing 18000, or min_ring < 1). */
int32_t msc_gms_quiver(int32_t step_cdeg, int32_t min_ring, double* out, int32_t cap);
msc_status msc_gms_reach(msc_ctx* ctx, const msc_scene* scene, const msc_gms_arm* arm, const int32_t target[3],
                         int32_t want, int64_t* count_out, int32_t* sols_out, double* vec_out, int32_t* nsol_out);
/* The same search when only the first solutions are wanted (the reach pose of Step 3 is
 * the first): the segment-1 survivors are searched in order, in chunks (the first of
 * about 4*2^20 (survivor, segment-2 vector) pairs, each next one twice the last), and the
 * search stops after the chunk in which the solutions found reach `want`.  The outputs are those of msc_gms_reach (the same first
 * min(want, total) solutions, vectors and status), except that *count_out is the number
 * of solutions of the survivors searched, between min(want, total) and total. */
msc_status msc_gms_reach_first(msc_ctx* ctx, const msc_scene* scene, const msc_gms_arm* arm, const int32_t target[3],
                               int32_t want, int64_t* count_out, int32_t* sols_out, double* vec_out,
                               int32_t* nsol_out);

/* Forward-kinematics replay of `count` poses (poses_cdeg[count*dof]) on the GPU:
 * valid_out[i] = 1 if the base is free and every segment sample is inside the grid
 * and free, else 0; end_out[i*3..] = end voxel of the chain (computed even when
 * invalid).  end_out may be NULL. */
msc_status msc_pose_check(msc_ctx* ctx, const msc_scene* scene, const msc_arm* arm,
                          const int32_t* poses_cdeg, int64_t count, uint8_t* valid_out,
                          int32_t* end_out);

/* Exact end point of discrete poses ("Exact IK solution with discretized segment
 * mappings"), FP64 on the GPU.  The arm's last two segments must each have two DOF:
 * joints dof-4 .. dof-1 are a zero-length link, a link of the other kind (length L3 > 0),
 * a zero-length link, a link of the other kind (length L4 > 0); else MSC_E_ARG.  For
 * pose i (poses_cdeg[i*dof..], multiples of the step) and exact target point
 * targets[i*3..] (voxel units, voxel centres at integer coordinates): the first dof-4
 * joints keep their discrete angles; P = the continuous end of those segments; the
 * joint J between the last two segments becomes the point with |J - P| = L3 and
 * |target - J| = L4 in the plane through P, the target and the discrete pose's joint,
 * on that joint's side (the closing point nearest to it; if the discrete joint lies on
 * the line P-target, the plane through u x e, e the axis least aligned with u, is
 * taken).  angles_out[i*dof..] receives every joint's angle in degrees: discrete ones,
 * then the continuous increments of the last four joints (each yaw adds to the
 * azimuth, each pitch to the elevation), unwrapped next to the discrete values.
 * status_out[i] = 0 when refined, 1 when |target - P| is 0 or outside [|L3 - L4|,
 * L3 + L4] (the discrete angles are written).  Joint limits and obstacles are not
 * re-checked: the exact pose stays in the plane of the cleared discrete one.  All
 * arrays are host memory owned by the caller; count may be 0.  The kernel time of each
 * launch (up to 2^20 poses) is left for msc_get_timings. */
msc_status msc_refine(msc_ctx* ctx, const msc_arm* arm, const int32_t* poses_cdeg,
                      const double* targets, int64_t count, double* angles_out,
                      int32_t* status_out);

/* msc_refine for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * checks and results as msc_refine (bit-identical angles and statuses), but the device
 * staging of poses, targets, angles and statuses lives in a fixed buffer of
 * MSC_REFINE_STATIC_BYTES that the library holds on each device until the process ends,
 * not in the context's workspace: the call allocates nothing.  At most
 * msc_refine_static_max(dof) poses per call (about 33 000 at 8 DOF); a larger count
 * returns MSC_E_CAPACITY with a message and writes nothing.  Every context on a device
 * shares that device's buffer and the buffer keeps the last call's contents (every output
 * is rewritten by each call): calls that overlap on one device, from different contexts or
 * threads, race and must be serialised by the caller.  Not profiled (msc_get_timings). */
#define MSC_REFINE_STATIC_BYTES (4u << 20)
msc_status msc_refine_static(msc_ctx* ctx, const msc_arm* arm, const int32_t* poses_cdeg,
                             const double* targets, int64_t count, double* angles_out,
                             int32_t* status_out);
/* Largest count msc_refine_static takes for an arm of `dof` joints (0 for a bad dof). */
int64_t msc_refine_static_max(int32_t dof);

/* Worker lanes for msc_batch and the server.  The workspace, minus a region for the
 * shared segment tables, is split into 1 + nworkers equal windows: one for this
 * context's own calls, one per worker lane.  Each worker lane has its own HIP stream
 * (default priority) and host thread, so the stages of different queries overlap on
 * the device.  Not allowed while a batch or the server runs (E_STATE).  nworkers in
 * 0..64. */
msc_status msc_ctx_set_lanes(msc_ctx* ctx, int32_t nworkers);
/* Workspace bytes of one lane window (what one query may use). */
uint64_t msc_lane_bytes(msc_ctx* ctx);

/* One query of a batch or of the server.  The caller owns the struct and the arrays it
 * points to until the query completes. */
typedef struct {
    const msc_scene* scene;
    const msc_arm* arm;
    int32_t kind;                /* 0 = reach pose (msc_reach), 1 = reach + path (msc_path, or
                                    msc_replan when ref_cdeg is set), 2 = reach-pose-guided path
                                    (msc_guided_path), 3 = path between poses (msc_pose_path) */
    int32_t target[3];
    const int32_t* start_cdeg;   /* path: [dof] start pose */
    int32_t waypoints;           /* path: moves W */
    int32_t max_delta_cdeg;      /* path: max joint change per move */
    int32_t* out;                /* reach: [dof]; path: [(waypoints+1)*dof]; kinds 2, 3: as the
                                    path_out of msc_guided_path / msc_pose_path (centidegrees) */
    msc_status status;           /* written when the query completes */
    float latency_ms;            /* written: submission (server) or batch start to completion */
    const int32_t* ref_cdeg;     /* path: NULL, or the original path's [(waypoints+1)*dof] rows:
                                    the query is then solved as msc_replan */
    int64_t tick;                /* written: the logical tick of the scene grid the query was
                                    solved on (0 for a scene without moving obstacles) */
    int32_t execute_ticks;       /* server path queries: > 0 = once solved, the path executes on
                                    the server's logical clock, waypoint w reached w*execute_ticks
                                    ticks after it completed, and msc_server_step re-validates its
                                    remaining waypoints; 0 = not executed */
    int32_t replan_depth;        /* written by the server: 0 for a submitted query, 1 + that of the
                                    path it replaces for a replan issued by msc_server_step */
    char error[128];             /* written: the message when status < 0, else "" */
    const msc_arm* virtual_arm;  /* kind 3: the virtual arm of msc_pose_path */
    msc_track track;             /* kinds 2 and 3: tracking parameters (msc_track_default values) */
    int32_t rows;                /* written: path rows of kinds 2 and 3 */
} msc_query;

/* Batched execution: solve nq independent queries; every worker lane takes the next
 * unsolved query when it finishes one (with no worker lanes, the context's own lane
 * solves them in order).  Results are those of msc_reach / msc_path / msc_guided_path /
 * msc_pose_path for each query alone ("The procedure for IK solution": the searches of
 * independent targets run in parallel).  With MSC_FUSED_TRACK in opts->flags the
 * waypoint tracking of the kind 2 and 3 queries is deferred and run for all of them in
 * one persistent launch on the context's stream, one block per query, once every search
 * has finished (same results).  Returns MSC_OK once every query ran; per-query results
 * are in q[i].status. */
msc_status msc_batch(msc_ctx* ctx, msc_query* q, int32_t nq, const msc_opts* opts);

/* Autotuner of the launch shapes of the set kernels (forward and backward stage
 * expansions, the meet, D marking): "The procedure for IK solution" notes that Steps
 * 2A/2B can be parallelized in various ways; how work items map to threads (the grid
 * cap, i.e. items per thread, and the number of lanes that share one state) is chosen
 * here by measurement.  Every query of q[nq] is solved on the context's own lane once per
 * shape variant to warm up and twice more with every launch timed (HIP events); for each
 * (kernel, log2 of the launch's input states) seen, the variant with the least total time
 * is kept in the context (the default shape where nothing was measured).  Results do not
 * depend on the shapes (the sets are the same).  With cache_path (may be NULL) the choice
 * is written there as text, for msc_tune_load.  The queries' outputs are written as by
 * msc_batch.  E_STATE while the server runs; a query's error status is returned. */
msc_status msc_autotune(msc_ctx* ctx, msc_query* q, int32_t nq, const msc_opts* opts, const char* cache_path);
/* Loads a choice written by msc_autotune.  E_ARG for a file that is not one (or names
 * shapes this library does not have), E_STATE if it was tuned on another GPU model; the
 * context's choice is unchanged on error.  msc_ctx_create loads the file named by the
 * environment variable MSC_TUNE_CACHE when it exists and fits. */
msc_status msc_tune_load(msc_ctx* ctx, const char* cache_path);
/* The context's choice: up to cap entries (kernel, size class, variant, grid cap, lanes
 * change) into out[cap*5]; *count = number of entries. */
msc_status msc_tune_entries(msc_ctx* ctx, int32_t* out, int32_t cap, int32_t* count);

/* Device-memory estimate of one query (bytes), used for admission. */
uint64_t msc_query_bytes(const msc_query* q);

/* Server with continuous batching over the worker lanes (msc_ctx_set_lanes first).
 * Queries submitted while others run are admitted as lanes free up, their stages
 * overlapping on the device; each query is solved exactly as msc_reach / msc_path
 * would solve it alone (its scene fixes the obstacle grid of its logical tick).
 * submit returns E_NOMEM if the query's estimate exceeds a lane window and E_STATE if
 * the server is not running.  poll sets *done = 1 once q->status is written. */
msc_status msc_server_start(msc_ctx* ctx, const msc_opts* opts);
msc_status msc_server_submit(msc_ctx* ctx, msc_query* q, uint64_t* ticket);
/* Admission by queue depth ("Dynamic Obstacles": an answer is only useful while the
 * arm can still act on it): while max_pending submitted queries wait for a lane,
 * msc_server_submit refuses new ones with MSC_E_CAPACITY (no ticket, nothing queued),
 * so that the answers given stay timely under overload; 0 (the default when the server
 * starts) sets no limit.  Replans queued by msc_server_step are always admitted.
 * E_STATE if the server is not running, E_ARG if max_pending < 0. */
msc_status msc_server_set_limit(msc_ctx* ctx, int32_t max_pending);
/* *done = 1 once (and only the first time) the ticket's query has completed; E_STATE for
 * a ticket that was never issued or whose completion was already reported. */
msc_status msc_server_poll(msc_ctx* ctx, uint64_t ticket, int32_t* done);
/* Blocks until the ticket's query has completed; E_STATE as for msc_server_poll. */
msc_status msc_server_wait(msc_ctx* ctx, uint64_t ticket);
msc_status msc_server_stop(msc_ctx* ctx);

/* One logical tick of the server ("Dynamic Obstacles": a moving obstacle that will block
 * a waypoint ahead of the moving arm triggers a new path for the rest of the way, from
 * the current pose, with the least distance to the original path).  Call it after the
 * scenes' msc_scene_set_dynamic for the same tick.  For every path executing on the
 * server (msc_query.execute_ticks): the waypoint w reached at this tick is
 * (tick - completion tick) / execute_ticks; a path past its last waypoint is finished;
 * otherwise its waypoints w..W are re-validated on the scene's current grid (sampled
 * segment points free and in the grid, as msc_pose_check).  If they are all clear the
 * path goes on; if waypoint w itself is blocked the path stops (no pose to replan
 * from); else a replan (msc_replan semantics: start = waypoint w, W - w waypoints, the
 * same target, reference = waypoints w..W) is queued ahead of submitted queries and,
 * once solved, executes in its place.  The tick must not decrease.  report may be NULL. */
typedef struct {
    int32_t executing;      /* paths executing after the step */
    int32_t finished;       /* paths that passed their last waypoint */
    int32_t stopped;        /* paths whose current pose is blocked */
    int32_t replans;        /* replans queued */
    int64_t poses_checked;  /* waypoints re-validated */
} msc_step_report;
msc_status msc_server_step(msc_ctx* ctx, int64_t tick, msc_step_report* report);

/* Copies up to cap completed replans issued by msc_server_step into out (oldest first)
 * and sets *count.  Their pointers (arm, start_cdeg, out, ref_cdeg) point to storage the
 * server keeps until the next msc_server_take_replans or msc_server_stop; status,
 * tick, latency_ms (from the step that issued it) and replan_depth are filled. */
msc_status msc_server_take_replans(msc_ctx* ctx, msc_query* out, int32_t cap, int32_t* count);

/* Statistics of the last msc_reach / msc_path call on this context. */
typedef struct {
    int32_t split_m;                     /* split actually used */
    int32_t dof;
    int64_t fwd_count[MSC_MAX_DOF + 1];  /* |F_k|, k = 0..split_m */
    int64_t bwd_count[MSC_MAX_DOF + 1];  /* |B_k|, k = split_m..dof; -2 for the set the meet probes
                                            when it was built without a count (split >= 1 and no
                                            MSC_CAPTURE_SETS) */
    int64_t join_count;                  /* |C_m|; -1 when C_m was not built (split >= 1 without MSC_CAPTURE_SETS) */
    int32_t fwd_dense[MSC_MAX_DOF + 1];  /* 1 if F_k used a dense bitset, 0 if a hash set */
    int32_t bwd_dense[MSC_MAX_DOF + 1];
    int32_t attempts;                    /* path: (reach pose, radius) attempts in search order up to
                                            the returned one, all of them without a path (the
                                            library may have searched more at the same time) */
    int32_t tube_r;                      /* path: tube radius of the returned path */
    int32_t reach_index;                 /* path: index of the reach pose used (0 = first) */
} msc_stats;
msc_status msc_get_stats(msc_ctx* ctx, msc_stats* out);

/* Kernel launch records of the last call made with MSC_PROFILE, in launch order.  Each
 * launch is bracketed by two HIP events recorded on the context's stream. */
typedef enum {
    MSC_K_FILL = 0, MSC_K_TABLES, MSC_K_RASTER, MSC_K_ORIENT, MSC_K_SEED, MSC_K_EXPAND_FWD,
    MSC_K_EXPAND_BWD, MSC_K_COMPACT, MSC_K_JOIN, MSC_K_DMARK, MSC_K_DFS, MSC_K_POSE,
    MSC_K_TUBE_VALID, MSC_K_TUBE_SOLVE, MSC_K_REFINE, MSC_K_TRACK, MSC_K_COUNT
} msc_kernel;
typedef struct {
    int32_t kernel;     /* msc_kernel */
    int32_t stage;      /* stage produced (expansions), else -1 */
    int64_t in_count;   /* input states (expansions, compaction, join, marking), else 0 */
    int64_t out_count;  /* new states (expansions), survivors (join, marking), else 0 */
    float ms;           /* event-to-event duration */
    int64_t out_words;  /* expansions with MSC_COUNT_SETS: non-zero 64-bit words of the output set's
                           structure (dense words; hash slots holding a member) after the launch;
                           else -1 */
} msc_timing;
/* Copy up to cap records into out and set *count to the number recorded. */
msc_status msc_get_timings(msc_ctx* ctx, msc_timing* out, int32_t cap, int32_t* count);

/* Debug: the tables of segment `stage` of arm (0-based), as built on the device:
 * off[(ia*na + ie)*3 + c] = rounded segment offset, sweep[((ia*na + ie)*S + s)*3 + c]
 * = rounded sample point s+1 of S, na = 36000/step_cdeg. */
msc_status msc_debug_tables(msc_ctx* ctx, const msc_arm* arm, int32_t stage, int32_t* off,
                            int32_t* sweep);

/* Debug: copy the occupancy grid as one byte per voxel, index (z*n + y)*n + x, 1 = blocked. */
msc_status msc_debug_raster(msc_ctx* ctx, const msc_scene* scene, uint8_t* occ_out);

/* Debug: a stage set of the last msc_reach run with MSC_CAPTURE_SETS.  which: 0 = F_k
 * (forward, k <= split), 1 = B_k (backward, k >= split), 2 = C (join, stage ignored),
 * 3 = D_k (forward states on some solution).  Writes min(cap, size) keys, sorted
 * ascending, key = ((z*n + y)*n + x) << 16 | ia << 8 | ie, and *count = size. */
msc_status msc_debug_set(msc_ctx* ctx, int32_t which, int32_t stage, uint64_t* keys, uint64_t cap,
                         uint64_t* count);

/* Message of the last negative status on this context ("" if none). */
const char* msc_last_error(msc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MSC_H */
