"""The synthetic input recipe (no GPU): arms, scenes and queries of the workloads have
the sizes, ranges and structure the design states, are the same for the same seed, and
the path queries' targets are reachable by a walk of the stated length."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import synth


def test_arm_c2():
    a = synth.arm_c2()
    assert a.dof == 8 and a.lens == [30, 30, 25, 25, 20, 20, 15, 10]
    assert a.types == [synth.YAW, synth.PITCH] * 4
    assert a.lo_cdeg == [-17000] * 8 and a.hi_cdeg == [17000] * 8
    assert a.step_cdeg == 500 and a.na == 72 and a.base == (128, 128, 0)


def test_arm_c1_and_gms():
    a = synth.arm_c1()
    assert (a.dof, a.lens, a.step_cdeg, a.base) == (3, [10, 8, 6], 1000, (32, 32, 0))
    assert a.lo_cdeg == [0, -9000, -9000] and a.hi_cdeg == [35000, 9000, 9000]
    g = synth.arm_gms()
    assert g.dof == 8 and g.lens == [0, 60, 0, 50, 0, 40, 0, 25]
    assert g.types == [synth.YAW, synth.PITCH] * 4
    # the segment lengths are the 8-DOF chain's summed in pairs
    assert [g.lens[2 * i + 1] for i in range(4)] == [sum(synth.C2_LENS[2 * i:2 * i + 2]) for i in range(4)]


def column_voxels(base, height):
    return [(base[0], base[1], base[2] + h) for h in range(height + 1)]


def in_dilated_box(v, box, pad):
    lo, ext = box[:3], box[3:]
    return all(lo[a] - pad <= v[a] <= lo[a] + ext[a] - 1 + pad for a in range(3))


@pytest.mark.parametrize("seed", [0, 1, 5])
def test_scene_c2_recipe(seed):
    s = synth.scene_c2(seed)
    arm = synth.arm_c2()
    assert (s.n, s.dilate) == (256, 2)
    assert s.boxes.shape == (32, 6) and s.spheres.shape == (8, 4)
    lo, ext = s.boxes[:, :3], s.boxes[:, 3:]
    assert ext.min() >= 5 and ext.max() <= 40
    assert lo.min() >= 0 and (lo + ext).max() <= 256
    c, r = s.spheres[:, :3], s.spheres[:, 3]
    assert c.min() >= 0 and c.max() < 256 and r.min() >= 4 and r.max() <= 20
    # nothing, dilated, touches the column the first segment sweeps (it points up)
    col = column_voxels(arm.base, arm.lens[0])
    for b in s.boxes:
        assert not any(in_dilated_box(v, b, s.dilate) for v in col)
    for sp in s.spheres:
        cube = np.concatenate([sp[:3], [1, 1, 1]])
        assert not any(in_dilated_box(v, cube, int(sp[3]) + s.dilate) for v in col)


def test_scenes_are_seeded():
    a, b, c = synth.scene_c2(3), synth.scene_c2(3), synth.scene_c2(4)
    assert np.array_equal(a.boxes, b.boxes) and np.array_equal(a.spheres, b.spheres)
    assert not np.array_equal(a.boxes, c.boxes)


def test_scene_c1_recipe():
    s = synth.scene_c1(2)
    assert (s.n, s.dilate) == (64, 0) and s.boxes.shape == (4, 6) and s.spheres.shape == (0, 4)
    ext = s.boxes[:, 3:]
    assert ext.min() >= 3 and ext.max() <= 10


def permissive(end=(1, 2, 3)):
    """A pose function that accepts every pose."""
    def pf(q):
        q = np.asarray(q)
        return np.ones(len(q), bool), np.tile(np.asarray(end), (len(q), 1))
    return pf


@pytest.mark.parametrize("W,delta", [(16, 1), (5, 2), (1, 3)])
def test_walk_stays_in_its_window(W, delta):
    arm = synth.arm_c2()
    rng = synth.rng_for(99, W, delta)
    start = synth.candidate_poses(rng, arm, 1)[0]
    q, _ = synth.walk_target(rng, arm, start, W, delta, permissive())
    assert np.all(np.abs(q.astype(np.int64) - start) <= W * delta)
    assert np.all(q >= arm.lo_steps()) and np.all(q <= arm.hi_steps())


def test_walk_stays_put_when_every_move_is_refused():
    arm = synth.arm_c2()
    rng = synth.rng_for(98)
    start = synth.candidate_poses(rng, arm, 1)[0]

    def only_start(q):
        q = np.asarray(q)
        ok = np.all(q == start, axis=1)
        return ok, np.zeros((len(q), 3), np.int64)

    q, _ = synth.walk_target(rng, arm, start, 4, 1, only_start)
    assert np.array_equal(q, start)


def test_first_valid_pose_takes_the_first_accepted_draw():
    arm = synth.arm_c1()

    def odd_first_joint(q):
        q = np.asarray(q)
        return q[:, 0] % 2 == 1, q[:, :3]

    q, end, idx = synth.first_valid_pose(synth.rng_for(97), arm, odd_first_joint, batch=64)
    cand = synth.candidate_poses(synth.rng_for(97), arm, 64)
    first = int(np.flatnonzero(cand[:, 0] % 2 == 1)[0])
    assert idx == first and np.array_equal(q, cand[first]) and np.array_equal(end, cand[first, :3])


def test_query_c2_is_a_feasible_walk():
    """The start pose is valid on the scene and the target is the end voxel of a valid
    pose within start +- 16 steps (the walk's end)."""
    q = synth.query_c2(1, oracle.pose_fn_for)
    assert (q.waypoints, q.max_delta) == (16, 1) and q.seed == (2, 1)
    pf = oracle.pose_fn_for(q.arm, q.scene)
    valid, _ = pf(q.start[None, :].astype(np.int32))
    assert valid[0]
    _, end = synth.walk_target(synth.rng_for(2, 1, 2), q.arm, q.start, 16, 1, pf)
    assert tuple(int(v) for v in end) == q.target
    again = synth.query_c2(1, oracle.pose_fn_for)
    assert again.target == q.target and np.array_equal(again.start, q.start)
