"""GPU parity of the exact end point (msc_refine) with the oracle, through the C ABI:
random discrete poses of the two-DOF-per-segment arm with targets inside the end voxel,
the special cases, and the reach pose of a full-size query refined to a point of its
target voxel.  FP64 on both sides; the bar is 1e-9 degrees (the two sides round
trigonometric results independently)."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc, synth

from test_gpu_parity import say
from test_oracle_refine import fk_points

TOL = 1e-9


def compare(solver, arm, q, targets):
    ang, st = solver.refine(arm, q, targets)
    for i in range(len(q)):
        rst, rang = oracle.refine(arm, q[i], targets[i])
        assert st[i] == rst, (i, st[i], rst)
        assert np.abs(ang[i] - rang).max() < TOL, (i, ang[i], rang)
    return ang, st


@pytest.mark.gpu
@pytest.mark.parametrize("step", [500, 250, 1000])
def test_refine_random_poses(solver, step):
    arm = synth.arm_gms(step_cdeg=step)
    rng = synth.rng_for(909, step)
    q = synth.candidate_poses(rng, arm, 3000)
    s = arm.step_cdeg / 100.0
    ends = np.array([fk_points(arm, qi * s)[-1] for qi in q])
    targets = ends + rng.uniform(-0.5, 0.5, size=ends.shape)
    say("refine random", step)
    ang, st = compare(solver, arm, q, targets)
    assert (st == 0).mean() > 0.9


@pytest.mark.gpu
def test_refine_special_cases(solver):
    arm = synth.arm_gms()
    n = arm.dof
    s = arm.step_cdeg / 100.0
    rng = synth.rng_for(910, 0)
    q = synth.candidate_poses(rng, arm, 6)
    q[5] = 0
    q[5, 1] = 6                     # the last two segments in one line
    pts = [fk_points(arm, qi * s) for qi in q]
    L3, L4 = arm.lens[n - 3], arm.lens[n - 1]
    targets = np.array([
        pts[0][-1],                                             # exact discrete end
        pts[1][n - 4] + np.array([L3 + L4 + 0.25, 0.0, 0.0]),   # beyond reach
        pts[2][n - 4] + np.array([0.0, 0.0, abs(L3 - L4) - 0.25]),  # too near
        pts[3][n - 4],                                          # on P itself
        pts[4][-1] + np.array([0.5, -0.5, 0.5]),                # corner of the end voxel
        pts[5][n - 4] + (pts[5][-1] - pts[5][n - 4]) * 0.9,     # on the straight line
    ])
    ang, st = compare(solver, arm, q, targets)
    assert list(st) == [0, 1, 1, 1, 0, 0]
    assert np.abs(ang[0] - q[0] * s).max() < 1e-7


@pytest.mark.gpu
def test_refine_full_size_reach_pose(solver):
    q = synth.query_gms(1, solver.pose_fn_for)
    scene = solver.scene(q.scene)
    st, path = solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta)
    assert st == msc.OK
    pose = path[-1]
    rng = synth.rng_for(911, 0)
    targets = np.asarray(q.target, np.float64)[None, :] + rng.uniform(-0.5, 0.5, size=(64, 3))
    ang, rst = compare(solver, q.arm, np.repeat(pose[None, :], 64, axis=0), targets)
    assert (rst == 0).all()
    for i in range(64):
        assert np.abs(fk_points(q.arm, ang[i])[-1] - targets[i]).max() < 1e-9


@pytest.mark.gpu
def test_refine_rejects_arms_without_two_dof_segments(solver):
    with pytest.raises(msc.MscError):
        solver.refine(synth.arm_c2(), np.zeros((1, 8), np.int32), np.zeros((1, 3)))


@pytest.mark.gpu
def test_refine_rejects_non_finite_targets(solver):
    arm = synth.arm_gms()
    q = np.zeros((2, arm.dof), np.int32)
    t = np.array([[10.0, 10.0, 10.0], [np.nan, 0.0, 0.0]])
    with pytest.raises(msc.MscError):
        solver.refine(arm, q, t)
    ang, st = solver.refine(arm, q[:1], t[:1])
    assert ang.shape == (1, arm.dof)
