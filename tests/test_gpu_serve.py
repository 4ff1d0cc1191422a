"""Serving with dynamic obstacles: results in the mix equal results alone, and a moving
box driven onto the remaining waypoints of an executing path forces a replan."""
import numpy as np
import pytest

from paper_1906_10678_amd import msc, serve, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def solve_alone(solver, spec):
    arm = spec_arm(spec)
    if spec.kind == 0:
        return solver.reach(spec.scene, arm, list(spec.c.target))
    start = np.asarray(spec.start) // spec.step
    if spec.ref is not None:
        return solver.replan(spec.scene, arm, start, list(spec.c.target), spec.waypoints,
                             spec.c.max_delta_cdeg // spec.step, spec.ref // spec.step)
    return solver.path(spec.scene, arm, start, list(spec.c.target), spec.waypoints, spec.c.max_delta_cdeg // spec.step)


def spec_arm(spec):
    a = spec.arm_c
    n = a.dof
    return synth.Arm(types=list(a.type[:n]), lens=list(a.len_vox[:n]), lo_cdeg=list(a.lo_cdeg[:n]),
                     hi_cdeg=list(a.hi_cdeg[:n]), step_cdeg=a.step_cdeg, base=tuple(a.base), samples=a.samples,
                     az0_cdeg=a.az0_cdeg, el0_cdeg=a.el0_cdeg)


def test_serving_results_equal_alone(solver):
    solver.set_lanes(4)
    try:
        loop = serve.ServingLoop(solver, nscenes=4, seed=1, rate=60.0, keep_log=True, templates=40)
        rep = loop.run(seconds=1.0, warmup_s=0.2)
        say("serve summary", rep.summary())
        assert rep.served > 5
        checked = 0
        for kind, tick, st, res, spec in rep.done_log[:24]:
            est, eres = solve_alone(solver, spec)
            assert st == est, (kind, tick, st, est)
            if st == msc.OK:
                assert np.array_equal(res, eres)
            checked += 1
        assert checked > 0
    finally:
        solver.set_lanes(0)


def test_forced_replan(solver):
    """A box moved onto a remaining waypoint of an executing path triggers a replan from
    the current pose; the new path starts at the current pose, is clear of the box and
    ends on the same target (or the target is no longer reachable)."""
    from oracle import pose_joints, raster

    solver.set_lanes(2)
    try:
        for seed in range(3, 11):
            loop = serve.ServingLoop(solver, nscenes=1, seed=seed, rate=0.0, templates=1)
            loop.dyn[0].movers = []
            loop.advance_tick()
            arm = synth.arm_c2()
            scene = loop.grids[0][0]
            pf = lambda qq, sc=scene: solver.pose_check(sc, arm, qq)  # noqa: E731
            start, _, _ = synth.first_valid_pose(synth.rng_for(8, seed), arm, pf)
            _, target = synth.walk_target(synth.rng_for(8, seed, 1), arm, start, 16, 1, pf)
            st, path = solver.path(scene, arm, start, target, 16, 1)
            if st != msc.OK:
                continue
            occ = raster(loop.dyn[0].static)
            _, j0 = pose_joints(arm, occ, path[0])
            # the joint of a later waypoint farthest (Euclidean) from every joint of the
            # current pose; a single blocked voxel dilated by 2 must not touch the current pose
            best, where = 0.0, None
            for w in range(2, 16):
                _, jw = pose_joints(arm, occ, path[w])
                for p in jw[1:]:
                    dmin = np.sqrt(((j0 - p) ** 2).sum(axis=1)).min()
                    if dmin > best:
                        best, where = dmin, p
            if best <= 4.0:
                continue
            ex = serve.Executing(path=path, target=tuple(int(v) for v in target), arm=arm, scene_idx=0, start_tick=0)
            loop.executing = [ex]
            loop.dyn[0].movers = [serve.MovingBox(pos=np.asarray(where, np.int64) * serve.FIX,
                                                  vel=np.zeros(3, np.int64), ext=np.ones(3, np.int64))]
            solver.server_start()
            try:
                loop.tick = 1
                loop.advance_tick()
                loop.revalidate()
                if loop.report.replans == 0:
                    continue  # the voxel also hit the current pose's segments
                assert len(loop.pending) == 1
                req = loop.pending[0]
                st2, new_path, _ = solver.wait(req.ticket)
                loop.pending = []
                say("replan status", st2)
                if st2 == msc.OK:
                    assert np.array_equal(new_path[0], path[0])
                    valid, ends = solver.pose_check(loop.grids[1][0], arm, new_path)
                    assert valid.all() and tuple(ends[-1]) == tuple(int(v) for v in target)
                else:
                    assert st2 in (msc.NO_REACH, msc.NO_PATH)
                return
            finally:
                solver.server_stop()
        pytest.fail("no seed produced a replan")
    finally:
        solver.set_lanes(0)
