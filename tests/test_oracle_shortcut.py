"""Pins of the oracle's short-reach shortcut ("Short Reaches").

* The shortcut is checked against a brute-force enumeration: every joint prefix
  (q_1..q_k), k = 2..K, inside the limits, in the canonical order (joint 1 first, each
  joint by |a| then a), whose segments 1..k-1 replay clear (pose_joints of the prefix
  arm, no pruning), with segment k's samples taken from the tables; the least (length,
  squared distance, k) and the first prefix that has it.
* The returned hit is replayed on its own: the hit point is the tuple's segment-k sample
  s, within the radius of the target, with every earlier sample free.
* The path: every row valid, joint changes within the relaxed filter, the end effector
  within the tolerance of the shortcut's waypoints, the reach pose last; without a hit
  the path is the reach-pose-guided path.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import guided, shortcut
from paper_1906_10678_amd import synth

from cases import tiny_case


def wide(arm):
    na = 36000 // arm.step_cdeg
    arm.lo_cdeg = [-(na // 2 - 1) * arm.step_cdeg] * arm.dof
    arm.hi_cdeg = [(na // 2 - 1) * arm.step_cdeg] * arm.dof
    return arm


def brute_shortcut(arm, occ, target, rho2, K):
    na, S = 36000 // arm.step_cdeg, arm.samples
    lo, hi = guided.arm_lo(arm), guided.arm_hi(arm)
    N = occ.shape[0]
    best = None
    for k in range(2, K + 1):
        pre = guided.sub_arm(arm, k - 1)
        _, sweep = oracle.tables(na, S, arm.lens[k - 1])
        axes = [sorted(range(lo[j], hi[j] + 1), key=lambda a: (abs(a), a)) for j in range(k)]
        for q in itertools.product(*axes):
            ok, joints = oracle.pose_joints(pre, occ, q[:k - 1])
            if not ok:
                continue
            ia, ie = (arm.az0_cdeg // arm.step_cdeg) % na, (arm.el0_cdeg // arm.step_cdeg) % na
            for j in range(k):
                if arm.types[j] == 0:
                    ia = (ia + q[j]) % na
                else:
                    ie = (ie + q[j]) % na
            p = joints[k - 1]
            for s in range(S):
                pt = p + sweep[ia, ie, s]
                if (pt < 0).any() or (pt >= N).any() or occ[pt[2], pt[1], pt[0]]:
                    break
                d2 = int(((pt - np.asarray(target)) ** 2).sum())
                if d2 <= rho2:
                    key = (S * sum(arm.lens[:k - 1]) + (s + 1) * arm.lens[k - 1], d2, k)
                    if best is None or key < best[0]:
                        best = (key, q, s + 1)
                    break
    return best


def cases(seeds, dof=4):
    for seed in seeds:
        arm, sc, rng = tiny_case(seed, dof=dof)
        arm = wide(arm)
        occ = oracle.raster(sc)
        q = synth.candidate_poses(rng, arm, 300)
        ok, ends = oracle.poses(arm, occ, q)
        for i in np.flatnonzero(ok)[:2]:
            pts = guided.sample_points(arm, q[i])
            # targets on and next to the pose's own segments 2 and 3 (hits), and its end
            for t in (pts[1][arm.samples // 2], pts[2][1] + np.array([0, 1, 0]), ends[i]):
                yield arm, occ, np.asarray(t, np.int64)


@pytest.mark.parametrize("rho2", [0, 1])
def test_shortcut_matches_enumeration(rho2):
    K = 3
    checked = hits = 0
    for arm, occ, t in cases(range(6)):
        if not shortcut.check_radius(arm, rho2, K) or occ[t[2], t[1], t[0]]:
            continue
        r = oracle.reach(arm, occ, t, m=K - 1, want=1, keep_sets=True)
        if r.status != oracle.OK:
            continue
        got = shortcut.shortcut(arm, occ, t, rho2, K, r.sets)
        want = brute_shortcut(arm, occ, t, rho2, K)
        checked += 1
        if want is None:
            assert got is None
            continue
        hits += 1
        (length, d2, k), q, s = want
        assert got is not None
        assert (got["length"], got["d2"], got["k"], got["s"]) == (length, d2, k, s)
        assert tuple(got["q"]) == tuple(q), (got["q"], q)
    assert checked >= 10 and hits >= 5


def test_hit_replays_on_its_own():
    for arm, occ, t in cases(range(4)):
        rho2, K = 1, 3
        if not shortcut.check_radius(arm, rho2, K) or occ[t[2], t[1], t[0]]:
            continue
        r = oracle.reach(arm, occ, t, m=K - 1, keep_sets=True)
        if r.status != oracle.OK:
            continue
        hit = shortcut.shortcut(arm, occ, t, rho2, K, r.sets)
        if hit is None:
            continue
        k, s = hit["k"], hit["s"]
        pts = guided.sample_points(guided.sub_arm(arm, k), hit["q"])
        ok, _ = oracle.pose_joints(guided.sub_arm(arm, k - 1), occ, hit["q"][:k - 1])
        assert ok
        for i in range(s):
            p = pts[k - 1][i]
            assert occ[p[2], p[1], p[0]] == 0
        assert np.array_equal(pts[k - 1][s - 1], hit["point"])
        assert int(((hit["point"] - t) ** 2).sum()) == hit["d2"] <= rho2
        for i in range(s - 1):
            assert int(((pts[k - 1][i] - t) ** 2).sum()) > rho2     # the first sample near the target


def test_short_path_invariants():
    seen = {"hit": 0, "fallback": 0}
    for arm, occ, t in cases(range(8)):
        rho2, K = 1, 3
        if not shortcut.check_radius(arm, rho2, K) or occ[t[2], t[1], t[0]]:
            continue
        st, rows, hit, r = shortcut.short_path(arm, occ, t, rho2, K, None, 1, 2, 4, retries=3)
        if st == oracle.NO_REACH:
            continue
        if hit is None:
            gst, grows, gr = guided.guided_path(arm, occ, t, None, 1, 2, 4, retries=3, m=K - 1)
            assert gst == st and (st != oracle.OK or np.array_equal(rows, grows))
            seen["fallback"] += 1
            continue
        if st != oracle.OK:
            continue
        seen["hit"] += 1
        pts = shortcut.shortcut_waypoints(arm, hit)
        assert np.array_equal(rows[-1], r.sols[r.index])
        back = rows[::-1]
        ok, ends = oracle.poses(arm, occ, back)
        assert ok.all()
        assert np.abs(np.diff(back.astype(np.int64), axis=0)).max(initial=0) <= 2
        assert (((ends[1:] - pts) ** 2).sum(axis=1) <= 4).all()
        assert np.array_equal(ends[0], t)
    assert seen["hit"] >= 3


def test_collision_before_the_hit_point_counts():
    """A voxel blocked on a pose's segment 2, before the sample chosen as the target: the
    hypothesis along that segment passes the obstacle before it comes near the target,
    so it is no hit.  The oracle agrees with the enumeration (which checks the samples
    before the hit), and in some of these cases a search that skipped that check would
    answer otherwise."""
    differs = checked = 0
    for seed in range(8):
        arm, sc, rng = tiny_case(seed, dof=4, nbox=0, nsph=0)
        arm = wide(arm)
        q = synth.candidate_poses(rng, arm, 200)
        occ0 = oracle.raster(sc)
        ok, _ = oracle.poses(arm, occ0, q)
        for i in np.flatnonzero(ok)[:3]:
            pts = guided.sample_points(arm, q[i])
            t, blk = pts[1][5], pts[1][2]
            if np.array_equal(t, blk) or np.array_equal(blk, pts[0][arm.samples - 1]):
                continue
            occ = occ0.copy()
            occ[blk[2], blk[1], blk[0]] = 1
            rho2, K = 1, 3
            if not shortcut.check_radius(arm, rho2, K):
                continue
            r = oracle.reach(arm, occ, t, m=K - 1, keep_sets=True)
            if r.status != oracle.OK:
                continue
            got = shortcut.shortcut(arm, occ, t, rho2, K, r.sets)
            want = brute_shortcut(arm, occ, t, rho2, K)
            checked += 1
            assert (got is None) == (want is None)
            if want is not None:
                assert (got["length"], got["d2"], got["k"], got["s"], tuple(got["q"])) == \
                    (want[0][0], want[0][1], want[0][2], want[2], tuple(want[1]))
            loose = brute_shortcut(arm, occ0, t, rho2, K)   # the obstacle ignored
            differs += (loose is None) != (want is None) or (loose is not None and loose[:2] != want[:2])
    assert checked >= 5 and differs >= 1
