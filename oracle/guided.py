"""Oracle of the workspace-guided paths: the reach-pose-guided path and the path between
arbitrary poses through a virtual arm.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the GPU library or its
binding.  It shares no code with the GPU path; it builds on the oracle's pinned pose
replay, tables and staged reach search.  Plain numpy; joint values are integer steps.

The paper's method ("Path Planning", "Smooth sequence computation", "Filtering for
smoothness", "Path between Arbitrary Poses"), in this discrete model:

* Waypoints are collision sample points of a solution already found.  For the
  reach-pose-guided path they are the sample points of the reach pose's segments
  ``tracked .. 2`` walked from the distal end toward the root, ending at the end of
  segment 1, the root of the moving part of the arm (segment 1 rises from the base
  along the initial orientation and its joint only spins it).  The joint that follows
  them is the end of the first ``tracked`` segments: 6 of 8 joints by default, the
  paper's 6-DOF sub-arm whose distal end traverses the path while the last segment is
  carried along.  For a path between arbitrary poses they are the
  sample points of a virtual arm rooted at the start pose's tracked joint and reaching
  for the target, walked from its root outward.
* The sequence is built one waypoint at a time from the previous pose (backward from
  the reach pose, resp. forward from the start pose).  The pose at a waypoint is, among
  the poses within ``delta`` steps of the previous one in every joint (the smoothness
  filter as a bound on the change of joint angle per waypoint) that are clear of
  obstacles and put the tracked joint within ``eps2`` (squared voxels) of the waypoint
  (a tolerance larger than the reach pose's, "Smooth sequence computation"), the one
  closest in configuration: smallest L1 joint change, then smallest squared distance
  to the waypoint, then the canonical order of the reach search centred on the previous
  pose (per joint (|change|, change), joint 1 first).
* When no pose qualifies, the filter is relaxed to ``delta2`` for that waypoint only
  (adaptive relaxation after a failure); when that fails too, the next solution of the
  reach search in the canonical order is tried (Step 3: another reach pose), up to
  ``retries``.

Parity status: pinned in tests/test_oracle_guided.py against a brute-force enumeration
of the filtered box in canonical order (built from pose_joints, not from this module's
replay), closed-form bounds of the waypoints, special cases (a tolerance that keeps the
previous pose, a zero filter that relaxes to the same sequence), and invariants of every
returned path.
"""
from __future__ import annotations

from types import SimpleNamespace
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import NO_PATH, NO_REACH, OK, poses, reach, tables


def sub_arm(arm, tracked: int):
    """The first ``tracked`` joints and segments of an arm (same base and limits)."""
    return SimpleNamespace(types=list(arm.types[:tracked]), lens=list(arm.lens[:tracked]),
                           lo_cdeg=list(arm.lo_cdeg[:tracked]), hi_cdeg=list(arm.hi_cdeg[:tracked]),
                           step_cdeg=arm.step_cdeg, base=tuple(arm.base), samples=arm.samples,
                           az0_cdeg=arm.az0_cdeg, el0_cdeg=arm.el0_cdeg)


def rooted(arm, base: Sequence[int]):
    """The same arm with another base voxel."""
    return SimpleNamespace(types=list(arm.types), lens=list(arm.lens), lo_cdeg=list(arm.lo_cdeg),
                           hi_cdeg=list(arm.hi_cdeg), step_cdeg=arm.step_cdeg,
                           base=tuple(int(v) for v in base), samples=arm.samples, az0_cdeg=arm.az0_cdeg,
                           el0_cdeg=arm.el0_cdeg)


def sample_points(arm, q: Sequence[int]) -> List[List[np.ndarray]]:
    """Collision sample points of pose q: pts[k][s-1] = p_{k-1} + sweep_k[o_k][s], s = 1..S
    (the last is the segment's end p_k), for every segment k = 1..n."""
    na, S = 36000 // arm.step_cdeg, arm.samples
    ia, ie = (arm.az0_cdeg // arm.step_cdeg) % na, (arm.el0_cdeg // arm.step_cdeg) % na
    p = np.array(arm.base, np.int64)
    out = []
    for k in range(len(arm.types)):
        if arm.types[k] == 0:
            ia = (ia + int(q[k])) % na
        else:
            ie = (ie + int(q[k])) % na
        _, sweep = tables(na, S, arm.lens[k])
        out.append([p + sweep[ia, ie, s].astype(np.int64) for s in range(S)])
        p = p + sweep[ia, ie, S - 1].astype(np.int64)
    return out


def reach_waypoints(arm, q_reach: Sequence[int], tracked: int) -> np.ndarray:
    """Waypoints of the reach-pose-guided path, in the order they are visited going
    backward from the reach pose: the sample points of segments tracked..2 (segments of
    length 0 have none), each segment from its end toward its start, then the end p_1 of
    segment 1 (the root waypoint: segment 1 rises from the base along the initial
    orientation and its joint only turns it about that axis, so p_1 is where the moving
    part of the arm is rooted); the first point of that walk is the tracked joint of the
    reach pose itself and is left out.  (M, 3) with M = S * (segments of nonzero length
    among 2..tracked); none for tracked <= 1."""
    if tracked <= 1:
        return np.zeros((0, 3), np.int64)
    pts = sample_points(arm, q_reach)
    walk = []
    for k in range(tracked - 1, 0, -1):
        if arm.lens[k] == 0:
            continue
        walk.extend(pts[k][s] for s in range(arm.samples - 1, -1, -1))
    if not walk:
        return np.zeros((0, 3), np.int64)
    walk.append(pts[0][arm.samples - 1])
    return np.array(walk[1:], np.int64)


def virtual_waypoints(varm, v: Sequence[int]) -> np.ndarray:
    """Waypoints along a virtual arm's pose v, root outward: the sample points of its
    segments 1..V (length-0 segments have none), s = 1..S each; the last is its end."""
    pts = sample_points(varm, v)
    walk = [pts[k][s] for k in range(len(varm.types)) if varm.lens[k] > 0 for s in range(varm.samples)]
    return np.array(walk, np.int64).reshape(-1, 3)


def _box(q: np.ndarray, d: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    axes = [np.arange(max(q[k] - d, lo[k]), min(q[k] + d, hi[k]) + 1) for k in range(len(q))]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1).astype(np.int64)


def track_step(arm, occ: np.ndarray, q_prev: Sequence[int], point: Sequence[int], tracked: int, delta: int,
               eps2: int, lo=None, hi=None) -> Optional[np.ndarray]:
    """The pose at one waypoint: among the poses within ``delta`` of q_prev (and the
    limits) that are valid and put joint ``tracked`` within eps2 of ``point``, the one
    with the smallest (L1 change, squared distance, canonical order around q_prev)."""
    q_prev = np.asarray(q_prev, np.int64)
    lo = arm_lo(arm) if lo is None else np.asarray(lo, np.int64)
    hi = arm_hi(arm) if hi is None else np.asarray(hi, np.int64)
    cand = _box(q_prev, delta, lo, hi)
    valid, _ = poses(arm, occ, cand)
    if tracked > 0:
        _, ends = poses(sub_arm(arm, tracked), occ, cand[:, :tracked])
    else:
        ends = np.tile(np.array(arm.base, np.int64), (len(cand), 1))
    d2 = ((ends - np.asarray(point, np.int64)) ** 2).sum(axis=1)
    ok = valid & (d2 <= eps2)
    if not ok.any():
        return None
    cand, d2 = cand[ok], d2[ok]
    t = cand - q_prev
    l1 = np.abs(t).sum(axis=1)
    # np.lexsort: the last key is the primary one
    keys = []
    for k in range(len(q_prev) - 1, -1, -1):
        keys.append(t[:, k])
        keys.append(np.abs(t[:, k]))
    keys.append(d2)
    keys.append(l1)
    return cand[np.lexsort(keys)[0]]


def arm_lo(arm) -> np.ndarray:
    return np.array(arm.lo_cdeg, np.int64) // arm.step_cdeg


def arm_hi(arm) -> np.ndarray:
    return np.array(arm.hi_cdeg, np.int64) // arm.step_cdeg


def track(arm, occ, q0, points: np.ndarray, tracked: int, delta: int, delta2: int, eps2: int
          ) -> Tuple[Optional[np.ndarray], int]:
    """Follow the waypoints from q0: rows q_0 = q0, q_1 .. q_M, each from the previous by
    track_step with delta, relaxed to delta2 at a waypoint where delta finds nothing.
    Returns (rows, M) or (None, index of the waypoint that failed)."""
    rows = [np.asarray(q0, np.int64)]
    for w in range(len(points)):
        q = track_step(arm, occ, rows[-1], points[w], tracked, delta, eps2)
        if q is None and delta2 != delta:
            q = track_step(arm, occ, rows[-1], points[w], tracked, delta2, eps2)
        if q is None:
            return None, w
        rows.append(q)
    return np.array(rows, np.int64), len(points)


def guided_path(arm, occ, target, tracked: Optional[int] = None, delta: int = 1, delta2: int = 2, eps2: int = 9,
                retries: int = 4, m: Optional[int] = None, approach=None):
    """Reach-pose-guided path: (status, rows[(M+1), dof] from the root waypoint's pose to
    the reach pose, reach result).  The reach search is unwindowed with reference 0 (as
    a plain reach query); each of its first ``retries`` poses is tracked in turn."""
    n = len(arm.types)
    tracked = n - 2 if tracked is None else tracked
    r = reach(arm, occ, target, m=m, want=retries, keep_sets=False, approach=approach)
    if r.status != OK:
        return r.status, None, r
    for i in range(min(retries, len(r.sols))):
        qs = np.asarray(r.sols[i], np.int64)
        pts = reach_waypoints(arm, qs, tracked)
        rows, _ = track(arm, occ, qs, pts, tracked, delta, delta2, eps2)
        if rows is not None:
            r.index = i
            return OK, rows[::-1].astype(np.int32), r
    return NO_PATH, None, r


def pose_path(arm, occ, start, target, varm, tracked: Optional[int] = None, delta: int = 1, delta2: int = 2,
              eps2: int = 9, retries: int = 4, m: Optional[int] = None):
    """Path between arbitrary poses: a virtual arm ``varm`` rooted at the start pose's
    tracked joint (its own base is replaced) reaches for the target; the tracked joint
    of the real arm follows the sample points of each of the virtual arm's first
    ``retries`` reach poses in turn, forward from the start pose.  Returns (status,
    rows[(M+1), dof] with row 0 = start, virtual reach result); E_ARG-like None status
    is not produced here: the caller checks the start pose."""
    n = len(arm.types)
    tracked = n if tracked is None else tracked
    start = np.asarray(start, np.int64)
    if tracked > 0:
        _, ends = poses(sub_arm(arm, tracked), occ, start[None, :tracked])
        root = ends[0]
    else:
        root = np.array(arm.base, np.int64)
    va = rooted(varm, root)
    r = reach(va, occ, target, m=m, want=retries, keep_sets=False)
    if r.status != OK:
        return r.status, None, r
    for i in range(min(retries, len(r.sols))):
        pts = virtual_waypoints(va, r.sols[i])
        rows, _ = track(arm, occ, start, pts, tracked, delta, delta2, eps2)
        if rows is not None:
            r.index = i
            return OK, rows.astype(np.int32), r
    return NO_PATH, None, r
