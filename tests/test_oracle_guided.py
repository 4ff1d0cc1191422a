"""Pins of the oracle's workspace-guided paths ("Path Planning", "Smooth sequence
computation", "Filtering for smoothness", "Path between Arbitrary Poses").

* One waypoint step is an argmin over a finite box of poses; it is checked against a
  plain enumeration that walks the box in the canonical order (offsets per joint sorted
  by (|t|, t), joint 1 first) and keeps the first pose of smallest (L1 change, squared
  distance), replaying every pose with pose_joints (not the batch replay the oracle
  uses).
* Waypoints are checked against the continuous sample points of the segments (each
  within the half-voxel rounding bound of p_{k-1} + (s/S) L d(o_k)), their count, their
  order and their ends (joint voxels; the end of segment 1 last).
* Special cases: a tolerance that admits the previous pose keeps it at every waypoint;
  a zero filter relaxed to delta gives the sequence of the filter delta.
* Every returned path: valid poses, joint changes within the relaxed filter, the
  tracked joint within the tolerance of its waypoint, the reach pose (resp. the start)
  at the right end, and the reach poses tried in the canonical order.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import guided
from paper_1906_10678_amd import synth

from cases import tiny_case


def limits(arm):
    return guided.arm_lo(arm), guided.arm_hi(arm)


def brute_step(arm, occ, q_prev, point, tracked, d, eps2):
    lo, hi = limits(arm)
    offs = sorted(range(-d, d + 1), key=lambda t: (abs(t), t))
    best = None
    for combo in itertools.product(offs, repeat=len(q_prev)):
        q = np.asarray(q_prev, np.int64) + np.array(combo, np.int64)
        if (q < lo).any() or (q > hi).any():
            continue
        ok, joints = oracle.pose_joints(arm, occ, q)
        if not ok:
            continue
        d2 = int(((joints[tracked] - np.asarray(point)) ** 2).sum())
        if d2 > eps2:
            continue
        key = (int(np.abs(combo).sum()), d2)
        if best is None or key < best[0]:
            best = (key, q)
    return None if best is None else best[1]


def valid_poses(arm, occ, rng, count):
    q = synth.candidate_poses(rng, arm, 400)
    ok, _ = oracle.poses(arm, occ, q)
    return q[ok][:count]


@pytest.mark.parametrize("seed", range(8))
def test_track_step_matches_enumeration(seed):
    dof = 3 + seed % 2
    arm, scene, rng = tiny_case(seed, dof=dof)
    occ = oracle.raster(scene)
    qs = valid_poses(arm, occ, rng, 4)
    checked = 0
    for q in qs:
        _, joints = oracle.pose_joints(arm, occ, q)
        for tracked in range(0, dof + 1):
            for d, eps2 in ((1, 0), (1, 2), (2, 5), (1, 9)):
                point = joints[tracked] + rng.integers(-2, 3, size=3)
                got = guided.track_step(arm, occ, q, point, tracked, d, eps2)
                want = brute_step(arm, occ, q, point, tracked, d, eps2)
                if want is None:
                    assert got is None
                else:
                    assert got is not None and np.array_equal(got, want), (tracked, d, eps2)
                    checked += 1
    assert checked > 10


def test_track_step_order_separates_plausible_slips():
    """Cases where a smallest-distance-first order, or a canonical order that compares
    the last joint first, would pick another pose occur in the sample, so the
    enumeration pin above separates them."""
    diff_d2_first = diff_later_first = 0
    for seed in range(4):
        arm, scene, rng = tiny_case(seed, dof=3)
        occ = oracle.raster(scene)
        lo, hi = limits(arm)
        for q in valid_poses(arm, occ, rng, 4):
            _, joints = oracle.pose_joints(arm, occ, q)
            for tracked, off in itertools.product((1, 2, 3), ([1, 0, 0], [0, 1, 0], [0, 0, -1], [1, 0, 1])):
                # the pose itself just outside the tolerance: a move must win
                point = joints[tracked] + np.array(off)
                eps = int(np.sum(np.square(off))) - 1
                got = guided.track_step(arm, occ, q, point, tracked, 1, eps)
                if got is None:
                    continue
                cand = [np.asarray(q) + np.array(c) for c in itertools.product((-1, 0, 1), repeat=3)]
                cand = [c for c in cand if (c >= lo).all() and (c <= hi).all()]
                ok = [c for c in cand if oracle.pose_joints(arm, occ, c)[0]]
                d2 = lambda c: int(((oracle.pose_joints(arm, occ, c)[1][tracked] - point) ** 2).sum())
                ok = [c for c in ok if d2(c) <= eps]
                by_d2 = min(ok, key=lambda c: (d2(c), int(np.abs(c - q).sum()),
                                               tuple(x for t in (c - q) for x in (abs(t), t))))
                diff_d2_first += not np.array_equal(by_d2, got)
                later = min(ok, key=lambda c: (int(np.abs(c - q).sum()), d2(c),
                                               tuple(x for t in (c - q)[::-1] for x in (abs(t), t))))
                diff_later_first += not np.array_equal(later, got)
    assert diff_d2_first > 0 and diff_later_first > 0


def test_track_step_breaks_a_mirror_tie_toward_minus():
    """Two moves mirror each other about the waypoint: joint 1 (pitch) by -1 or +1 step
    puts the tracked joint at (8, 10, 3) or (12, 10, 3), both 8 squared voxels from
    (10, 10, 1), while the pose itself (joint at (10, 10, 4), 9 away) is outside the
    tolerance.  The canonical order takes -1 first."""
    arm = synth.Arm(types=[synth.PITCH, synth.YAW], lens=[4, 4], lo_cdeg=[-9000, -9000], hi_cdeg=[9000, 9000],
                    step_cdeg=3000, base=(10, 10, 0))
    occ = np.zeros((20, 20, 20), np.uint8)
    for j in (oracle.pose_joints(arm, occ, [-1, 0])[1], oracle.pose_joints(arm, occ, [1, 0])[1]):
        assert int(((j[1] - np.array([10, 10, 1])) ** 2).sum()) == 8
    got = guided.track_step(arm, occ, [0, 0], (10, 10, 1), 1, 1, 8)
    assert got.tolist() == [-1, 0]
    assert brute_step(arm, occ, [0, 0], (10, 10, 1), 1, 1, 8).tolist() == [-1, 0]


@pytest.mark.parametrize("seed", range(6))
def test_reach_waypoints_follow_the_segments(seed):
    arm, scene, rng = tiny_case(seed, dof=4)
    occ = oracle.raster(scene)
    S = arm.samples
    step = arm.step_cdeg / 100.0
    for q in valid_poses(arm, occ, rng, 3):
        ok, joints = oracle.pose_joints(arm, occ, q)
        assert ok
        for tracked in (2, 3, 4):
            pts = guided.reach_waypoints(arm, q, tracked)
            nz = sum(1 for k in range(1, tracked) if arm.lens[k] > 0)
            assert len(pts) == S * nz
            assert np.array_equal(pts[-1], joints[1])         # the end of segment 1 comes last
            # walk back: segment tracked first (its end is the start, left out)
            expect = []
            az, el = arm.az0_cdeg / 100.0, arm.el0_cdeg / 100.0
            dirs = []
            for k in range(arm.dof):
                if arm.types[k] == synth.YAW:
                    az += q[k] * step
                else:
                    el += q[k] * step
                a, e = math.radians(az), math.radians(el)
                dirs.append(np.array([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)]))
            for k in range(tracked - 1, 0, -1):
                for s in range(S, 0, -1):
                    expect.append((k, s))
            expect = expect[1:]
            for (k, s), p in zip(expect, pts[:-1]):
                cont = joints[k] + (s / S) * arm.lens[k] * dirs[k]
                assert np.abs(p - cont).max() <= 0.5 + 1e-9, (k, s)
                if s == S:
                    assert np.array_equal(p, joints[k + 1])
                assert occ[p[2], p[1], p[0]] == 0            # samples of a valid pose are free


def test_virtual_waypoints_end_on_the_virtual_pose():
    varm = synth.arm_virtual([4, 3, 0, 2], step_cdeg=3000, base=(10, 10, 5))
    rng = synth.rng_for(950, 0)
    occ = np.zeros((20, 20, 20), np.uint8)
    for v in synth.candidate_poses(rng, varm, 20):
        ok, joints = oracle.pose_joints(varm, occ, v)
        pts = guided.virtual_waypoints(varm, v)
        assert len(pts) == varm.samples * 3
        if ok:
            assert np.array_equal(pts[-1], joints[-1])
            assert np.array_equal(pts[varm.samples - 1], joints[2])   # end of the first segment


@pytest.mark.parametrize("seed", range(4))
def test_wide_tolerance_keeps_the_previous_pose(seed):
    arm, scene, rng = tiny_case(seed, dof=3)
    occ = oracle.raster(scene)
    q = valid_poses(arm, occ, rng, 1)[0]
    pts = guided.reach_waypoints(arm, q, 2)
    rows, m = guided.track(arm, occ, q, pts, 2, 1, 2, eps2=10 ** 6)
    assert m == len(pts) and (rows == np.asarray(q)).all()


@pytest.mark.parametrize("seed", range(6))
def test_zero_filter_relaxes_to_the_same_sequence(seed):
    arm, scene, rng = tiny_case(seed, dof=3)
    occ = oracle.raster(scene)
    for q in valid_poses(arm, occ, rng, 2):
        pts = guided.reach_waypoints(arm, q, 3)
        a, ma = guided.track(arm, occ, q, pts, 3, 0, 1, eps2=2)
        b, mb = guided.track(arm, occ, q, pts, 3, 1, 1, eps2=2)
        assert ma == mb
        assert (a is None) == (b is None)
        if a is not None:
            assert np.array_equal(a, b)
        # with no change allowed the tracked joint stays put: the walk stops at the
        # first waypoint farther than the tolerance from it
        c, mc = guided.track(arm, occ, q, pts, 3, 0, 0, eps2=2)
        _, joints = oracle.pose_joints(arm, occ, q)
        far = np.flatnonzero(((pts - joints[3]) ** 2).sum(axis=1) > 2)
        if far.size:
            assert c is None and mc == far[0]
        else:
            assert c is not None and (c == np.asarray(q)).all()


def check_rows(arm, occ, rows, pts, tracked, delta2, eps2):
    ok, _ = oracle.poses(arm, occ, rows)
    assert ok.all()
    assert np.abs(np.diff(rows.astype(np.int64), axis=0)).max(initial=0) <= delta2
    lo, hi = limits(arm)
    assert (rows >= lo).all() and (rows <= hi).all()
    if tracked > 0:
        _, ends = oracle.poses(guided.sub_arm(arm, tracked), occ, rows[:, :tracked])
    else:
        ends = np.tile(np.array(arm.base), (len(rows), 1))
    assert (((ends[1:] - pts) ** 2).sum(axis=1) <= eps2).all()


def wide(arm):
    """The same arm with every joint free over (-180, 180) degrees: room to fold."""
    na = 36000 // arm.step_cdeg
    arm.lo_cdeg = [-(na // 2 - 1) * arm.step_cdeg] * arm.dof
    arm.hi_cdeg = [(na // 2 - 1) * arm.step_cdeg] * arm.dof
    return arm


def guided_case(seed):
    dof = 3 + seed % 2
    arm, scene, rng = tiny_case(seed, dof=dof)
    return wide(arm), scene, rng, dof


def test_guided_path_invariants_and_retry_order():
    outcomes = []
    for seed in range(8):
        arm, scene, rng, dof = guided_case(seed)
        occ = oracle.raster(scene)
        tracked = dof - 1 + seed % 2
        for q in valid_poses(arm, occ, rng, 3):
            _, end = oracle.poses(arm, occ, q[None])
            st, rows, r = guided.guided_path(arm, occ, end[0], tracked, 1, 2, 4, retries=3)
            outcomes.append(st)
            assert st in (oracle.OK, oracle.NO_PATH)
            # the same reach poses, tracked by hand in the canonical order
            first = None
            for i in range(min(3, len(r.sols))):
                pts = guided.reach_waypoints(arm, r.sols[i], tracked)
                rr, _ = guided.track(arm, occ, r.sols[i], pts, tracked, 1, 2, 4)
                if rr is not None:
                    first = (i, rr, pts)
                    break
            if first is None:
                assert st == oracle.NO_PATH
                continue
            i, rr, pts = first
            assert st == oracle.OK and r.index == i
            assert np.array_equal(rows, rr[::-1])
            assert np.array_equal(rows[-1], r.sols[i])
            check_rows(arm, occ, rows[::-1], pts, tracked, 2, 4)
            # the first row puts the tracked joint near the root waypoint (end of segment 1)
            _, joints = oracle.pose_joints(arm, occ, rows[0])
            assert int(((joints[tracked] - pts[-1]) ** 2).sum()) <= 4
    assert outcomes.count(oracle.OK) >= 6 and oracle.NO_PATH in outcomes


def test_pose_path_invariants():
    seen_ok = 0
    for seed in range(6):
        seen_ok += _pose_path_case(seed)
    assert seen_ok >= 3


def _pose_path_case(seed):
    arm, scene, rng = tiny_case(seed, dof=3)
    arm = wide(arm)
    occ = oracle.raster(scene)
    varm = synth.arm_virtual([3, 3], step_cdeg=3000)
    qs = valid_poses(arm, occ, rng, 4)
    seen_ok = 0
    for a, b in zip(qs[:-1], qs[1:]):
        _, end = oracle.poses(arm, occ, b[None])
        st, rows, r = guided.pose_path(arm, occ, a, end[0], varm, None, 1, 2, 2, retries=3)
        if st == oracle.NO_REACH:
            continue
        if st == oracle.OK:
            seen_ok += 1
            assert np.array_equal(rows[0], a)
            _, joints = oracle.pose_joints(arm, occ, a)
            va = guided.rooted(varm, joints[-1])
            pts = guided.virtual_waypoints(va, r.sols[r.index])
            assert np.array_equal(pts[-1], end[0])
            check_rows(arm, occ, rows, pts, arm.dof, 2, 2)
            for i in range(r.index):
                rr, _ = guided.track(arm, occ, a, guided.virtual_waypoints(va, r.sols[i]), arm.dof, 1, 2, 2)
                assert rr is None
    return seen_ok
