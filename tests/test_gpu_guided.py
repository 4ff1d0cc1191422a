"""GPU parity of the workspace-guided paths (msc_guided_path, msc_pose_path) with the
oracle, through the C ABI: status, rows and the reach pose used, element by element, on
tiny arms (every tracked joint), medium arms on 48^3 grids, and full-size 8-DOF queries
of the path workload with a virtual arm; argument errors.  Integer work: bit-exact."""
import numpy as np
import pytest

import oracle
from oracle import guided
from paper_1906_10678_amd import msc, synth

from cases import tiny_case
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def wide(arm):
    na = 36000 // arm.step_cdeg
    arm.lo_cdeg = [-(na // 2 - 1) * arm.step_cdeg] * arm.dof
    arm.hi_cdeg = [(na // 2 - 1) * arm.step_cdeg] * arm.dof
    return arm


def valid_poses(arm, occ, rng, count):
    q = synth.candidate_poses(rng, arm, 400)
    ok, _ = oracle.poses(arm, occ, q)
    return q[ok][:count]


def compare_guided(solver, scene, arm, occ, target, tracked, delta, delta2, eps2, retries=3):
    st, rows = solver.guided_path(scene, arm, target, tracked, delta, delta2, eps2, retries=retries)
    rst, rrows, r = guided.guided_path(arm, occ, target, tracked, delta, delta2, eps2, retries=retries)
    assert st == rst, (st, rst)
    if st == msc.OK:
        assert np.array_equal(rows, rrows), (rows, rrows)
        assert solver.stats()["reach_index"] == r.index
    return st


def test_guided_tiny_every_tracked_joint(solver):
    outcomes = []
    for seed in range(10):
        dof = 3 + seed % 3
        arm, sc, rng = tiny_case(seed, dof=dof)
        arm = wide(arm)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        for q in valid_poses(arm, occ, rng, 2):
            _, end = oracle.poses(arm, occ, q[None])
            for tracked in range(1, dof + 1):
                for delta, delta2, eps2 in ((1, 2, 4), (0, 1, 2), (1, 1, 9)):
                    say("guided tiny", seed, dof, tracked, delta, delta2, eps2)
                    outcomes.append(compare_guided(solver, scene, arm, occ, end[0], tracked, delta, delta2, eps2))
    assert outcomes.count(msc.OK) > 20 and msc.NO_PATH in outcomes


def test_guided_medium(solver):
    outcomes = []
    for seed in range(4):
        rng = synth.rng_for(960, seed)
        n = 48
        arm = synth.arm_chain(6, [8, 8, 7, 6, 5, 4], 1000, 17000, (n // 2, n // 2, 0))
        sc = synth.random_scene(rng, n, 1, 6, (3, 10), 2, (2, 5), base=arm.base, column=arm.lens[0] + 2)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        for q in valid_poses(arm, occ, rng, 2):
            _, end = oracle.poses(arm, occ, q[None])
            say("guided medium", seed)
            outcomes.append(compare_guided(solver, scene, arm, occ, end[0], 4, 1, 2, 9))
    assert msc.OK in outcomes


def test_guided_no_reach(solver):
    arm, sc, rng = tiny_case(1, dof=3)
    occ = oracle.raster(sc)
    scene = solver.scene(sc)
    blocked = np.argwhere(occ)
    if len(blocked) == 0:
        pytest.skip("scene without obstacles")
    z, y, x = blocked[0]
    st, rows = solver.guided_path(scene, arm, (x, y, z), 2, 1, 2, 4)
    assert st == msc.NO_REACH and rows is None


def compare_pose_path(solver, scene, arm, occ, start, target, varm, tracked, delta, delta2, eps2, retries=3):
    st, rows = solver.pose_path(scene, arm, start, target, varm, tracked, delta, delta2, eps2, retries=retries)
    rst, rrows, r = guided.pose_path(arm, occ, start, target, varm, tracked, delta, delta2, eps2, retries=retries)
    assert st == rst, (st, rst)
    if st == msc.OK:
        assert np.array_equal(rows, rrows)
        assert solver.stats()["reach_index"] == r.index
    return st


def test_pose_path_tiny(solver):
    outcomes = []
    for seed in range(10):
        dof = 3 + seed % 2
        arm, sc, rng = tiny_case(seed, dof=dof)
        arm = wide(arm)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        varm = synth.arm_virtual([3, 3], step_cdeg=arm.step_cdeg)
        qs = valid_poses(arm, occ, rng, 4)
        for a, b in zip(qs[:-1], qs[1:]):
            _, end = oracle.poses(arm, occ, b[None])
            for tracked in (dof, dof - 1):
                say("pose path tiny", seed, dof, tracked)
                outcomes.append(compare_pose_path(solver, scene, arm, occ, a, end[0], varm, tracked, 1, 2, 4))
    assert outcomes.count(msc.OK) > 5


def test_pose_path_full_size(solver):
    """8-DOF path workload queries: from the start pose to the target through a virtual
    arm of three 20-voxel segments, the end effector tracked."""
    outcomes = []
    for seed in range(4):
        q = synth.query_c2(seed, solver.pose_fn_for)
        occ = oracle.raster(q.scene)
        scene = solver.scene(q.scene)
        varm = synth.arm_virtual([20, 20, 20])
        say("pose path full size", seed)
        outcomes.append(compare_pose_path(solver, scene, q.arm, occ, q.start, q.target, varm, 8, 1, 2, 9))
    assert msc.OK in outcomes


def test_track_argument_errors(solver):
    arm, sc, rng = tiny_case(2, dof=3)
    scene = solver.scene(sc)
    occ = oracle.raster(sc)
    q = valid_poses(arm, occ, rng, 1)[0]
    _, end = oracle.poses(arm, occ, q[None])
    for kw in (dict(tracked=4), dict(tracked=0), dict(delta=2, delta2=1), dict(eps2=1024)):
        with pytest.raises(msc.MscError) as e:
            solver.guided_path(scene, arm, end[0], **kw)
        assert e.value.status == msc.E_ARG
    varm = synth.arm_virtual([3, 3], step_cdeg=1500)
    with pytest.raises(msc.MscError) as e:
        solver.pose_path(scene, arm, q, end[0], varm)
    assert e.value.status == msc.E_ARG and "step" in str(e.value)
    bad = synth.candidate_poses(rng, arm, 400)
    ok, _ = oracle.poses(arm, occ, bad)
    if (~ok).any():
        with pytest.raises(msc.MscError) as e:
            solver.pose_path(scene, arm, bad[~ok][0], end[0], synth.arm_virtual([3, 3], step_cdeg=arm.step_cdeg))
        assert e.value.status == msc.E_ARG


def test_batched_guided_and_pose_paths_equal_alone(solver):
    """Kinds 2 and 3 through msc_batch, mixed with plain reach queries, on 0 and 3
    worker lanes, with the tracking per lane and fused into one launch: every result is
    the query's alone (which the tests above compare with the oracle)."""
    specs_alone = []
    for seed in range(6):
        dof = 3 + seed % 2
        arm, sc, rng = tiny_case(seed, dof=dof)
        arm = wide(arm)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        varm = synth.arm_virtual([3, 3], step_cdeg=arm.step_cdeg)
        qs = valid_poses(arm, occ, rng, 3)
        for a, b in zip(qs[:-1], qs[1:]):
            _, end = oracle.poses(arm, occ, b[None])
            st, rows = solver.guided_path(scene, arm, end[0], dof - 1, 1, 2, 4)
            specs_alone.append((dict(scene=scene, arm=arm, target=end[0], kind=2, track=(dof - 1, 1, 2, 4)),
                                (st, rows)))
            st, rows = solver.pose_path(scene, arm, a, end[0], varm, dof, 1, 2, 4)
            specs_alone.append((dict(scene=scene, arm=arm, target=end[0], start=a, kind=3, virtual_arm=varm,
                                     track=(dof, 1, 2, 4)), (st, rows)))
            st, pose = solver.reach(scene, arm, end[0])
            specs_alone.append((dict(scene=scene, arm=arm, target=end[0]), (st, pose)))
    assert any(a[1][0] == msc.OK for a in specs_alone if a[0].get("kind") == 2)
    for lanes in (0, 3):
        for flags in (0, msc.FUSED_TRACK):
            say("batch guided lanes", lanes, "flags", flags)
            solver.set_lanes(lanes)
            try:
                specs = [msc.QuerySpec(**kw) for kw, _ in specs_alone]
                res = solver.batch(specs, flags=flags)
            finally:
                solver.set_lanes(0)
            for (kw, (st, val)), (bst, bval, _) in zip(specs_alone, res):
                assert bst == st, (kw.get("kind"), bst, st)
                if st == msc.OK:
                    assert np.array_equal(bval, val)
