"""Pins of the oracle on the paper's own arm model: two degrees of freedom per segment
(azimuth and elevation at the segment's proximal end, "Joint Angular Velocities"; eight
DOF = four segments, "The selection process for an 8DOF arm").  In the global az/el
model a two-DOF segment is a zero-length yaw link followed by the pitch joint that
carries the segment.  A zero-length link moves nothing and sweeps nothing, so the staged
search must treat it as a pure change of orientation: checked against exhaustive
enumeration on tiny arms, against its neutrality when its window is {0}, and against
the merge of two consecutive joints of the same kind.
"""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import synth

from cases import tiny_gms_case


def pick_target(arm, rng, occ, reachable=True):
    q = synth.candidate_poses(rng, arm, 256)
    if not reachable:
        return tuple(int(v) for v in rng.integers(0, occ.shape[0], size=3))
    valid, ends = oracle.poses(arm, occ, q)
    i = int(np.flatnonzero(valid)[0]) if valid.any() else 0
    return tuple(int(v) for v in ends[i])


GMS = [(s, segs, step) for s in range(6) for segs, step in [(2, 3000), (2, 4500), (3, 4500)]]


@pytest.mark.parametrize("seed,segs,step", GMS)
def test_gms_canonical_pose_matches_brute_force(seed, segs, step):
    arm, scene, rng = tiny_gms_case(seed, segs, step)
    occ = oracle.raster(scene)
    target = pick_target(arm, rng, occ, reachable=(seed % 3 != 2))
    cnt, sols = oracle.brute_solutions(arm, occ, target, cap=4)
    for m in range(arm.dof + 1):
        r = oracle.reach(arm, occ, target, m=m, want=4)
        assert (r.status == oracle.OK) == (cnt > 0), m
        assert np.array_equal(r.sols, sols), (m, r.sols, sols)


@pytest.mark.parametrize("seed,segs,step", GMS[:9])
@pytest.mark.parametrize("prune", [True, False])
def test_gms_stage_sets_match_enumeration(seed, segs, step, prune):
    arm, scene, rng = tiny_gms_case(seed, segs, step)
    occ = oracle.raster(scene)
    target = pick_target(arm, rng, occ)
    brute = oracle.brute_sets(arm, occ, target, kf=arm.dof, kb=0, prune=prune)
    for m in range(arm.dof + 1):
        r = oracle.reach(arm, occ, target, m=m, prune=prune)
        for k in range(m + 1):
            assert np.array_equal(r.sets[("F", k)], brute[("F", k)]), ("F", k, m)
        for k in range(m, arm.dof + 1):
            assert np.array_equal(r.sets[("B", k)], brute[("B", k)]), ("B", k, m)


@pytest.mark.parametrize("seed", range(6))
def test_zero_length_link_leaves_position(seed):
    """Every state after a zero-length link sits on a voxel of the stage before it, and
    every orientation its window allows is there (pruning off, no obstacles hit)."""
    arm, scene, rng = tiny_gms_case(seed, 2, 3000)
    occ = oracle.raster(scene)
    target = pick_target(arm, rng, occ)
    r = oracle.reach(arm, occ, target, m=arm.dof, prune=False)
    n = occ.shape[0]
    for k in range(0, arm.dof, 2):          # joint k (0-based) is a zero-length yaw link
        x0, y0, z0, ia0, ie0 = oracle.key_fields(r.sets[("F", k)], n)
        x1, y1, z1, ia1, ie1 = oracle.key_fields(r.sets[("F", k + 1)], n)
        before = set(zip(x0.tolist(), y0.tolist(), z0.tolist()))
        after = set(zip(x1.tolist(), y1.tolist(), z1.tolist()))
        assert after == before, k
        lo, hi = arm.lo_steps()[k], arm.hi_steps()[k]
        na = arm.na
        want = {(x, y, z, (ia + a) % na, ie) for x, y, z, ia, ie in
                zip(x0.tolist(), y0.tolist(), z0.tolist(), ia0.tolist(), ie0.tolist()) for a in range(lo, hi + 1)}
        got = set(zip(x1.tolist(), y1.tolist(), z1.tolist(), ia1.tolist(), ie1.tolist()))
        assert got == want, k


@pytest.mark.parametrize("seed", range(8))
def test_fixed_zero_length_link_is_neutral(seed):
    """A zero-length yaw link whose window is {0} inserted before every pitch joint of a
    chain changes nothing: same status, and the canonical poses with 0 inserted."""
    from cases import tiny_case
    arm, scene, rng = tiny_case(seed, 4, 3000)
    occ = oracle.raster(scene)
    target = pick_target(arm, rng, occ, reachable=(seed % 3 != 2))
    types, lens, lo, hi, pos = [], [], [], [], []
    for k in range(arm.dof):
        if arm.types[k] == synth.PITCH:
            types.append(synth.YAW), lens.append(0), lo.append(0), hi.append(0)
        pos.append(len(types))
        types.append(arm.types[k]), lens.append(arm.lens[k]), lo.append(arm.lo_cdeg[k]), hi.append(arm.hi_cdeg[k])
    arm2 = synth.Arm(types=types, lens=lens, lo_cdeg=lo, hi_cdeg=hi, step_cdeg=arm.step_cdeg, base=arm.base)
    r1 = oracle.reach(arm, occ, target, want=5, keep_sets=False)
    r2 = oracle.reach(arm2, occ, target, want=5, keep_sets=False)
    assert r1.status == r2.status
    assert np.array_equal(r2.sols[:, pos], r1.sols)
    assert not np.delete(r2.sols, pos, axis=1).any()


@pytest.mark.parametrize("seed", range(6))
def test_two_yaw_joints_merge(seed):
    """A zero-length yaw link with window A followed by a yaw joint with window B reaches
    the same states as one yaw joint with window A + B (Minkowski sum of the steps)."""
    step = 3000
    rng = synth.rng_for(907, seed)
    n = 20
    L1, L2 = [int(v) for v in rng.integers(2, 6, size=2)]
    a_lo, a_hi = sorted(int(v) for v in rng.integers(-3, 4, size=2))
    b_lo, b_hi = sorted(int(v) for v in rng.integers(-3, 4, size=2))
    p_lo, p_hi = sorted(int(v) for v in rng.integers(-4, 5, size=2))
    base = (n // 2, n // 2, 0)
    split = synth.Arm(types=[synth.PITCH, synth.YAW, synth.YAW], lens=[L1, 0, L2],
                      lo_cdeg=[p_lo * step, a_lo * step, b_lo * step], hi_cdeg=[p_hi * step, a_hi * step, b_hi * step],
                      step_cdeg=step, base=base)
    merged = synth.Arm(types=[synth.PITCH, synth.YAW], lens=[L1, L2],
                       lo_cdeg=[p_lo * step, (a_lo + b_lo) * step], hi_cdeg=[p_hi * step, (a_hi + b_hi) * step],
                       step_cdeg=step, base=base)
    scene = synth.random_scene(rng, n, 0, 3, (1, 5), 1, (1, 2), base=base, column=L1)
    occ = oracle.raster(scene)
    for t in range(4):
        target = tuple(int(v) for v in rng.integers(0, n, size=3))
        rs = oracle.reach(split, occ, target, m=3, prune=False)
        rm = oracle.reach(merged, occ, target, m=2, prune=False)
        assert np.array_equal(rs.sets[("F", 3)], rm.sets[("F", 2)])
        assert rs.status == rm.status
