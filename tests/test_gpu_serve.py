"""Serving with dynamic obstacles ("Dynamic Obstacles").

* The grid a scene holds for a tick equals the oracle's raster of the static plus the
  moving obstacles of that tick.
* Every request the server answered, and every replan it issued for an executing path,
  equals the oracle's answer on the grid of its tick, and the GPU's answer for the same
  query alone (served in the mix = solved alone).
* A box moved onto a later waypoint of an executing path makes the server replan the
  rest of the path from the current pose; the oracle checks the new path.
* Tickets of unknown or already reported queries are errors; an error's message is
  kept in the query record.
"""
import ctypes
import time

import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc, serve, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def small_arm(dof):
    """Arms of the 64^3 serving tests: short segments, 10 deg steps, +-170 deg."""
    return synth.arm_chain(dof, [10, 9, 8, 7, 6, 5, 4, 3], 1000, 17000, (32, 32, 0))


def spec_arm(spec):
    a = spec.arm_c
    n = a.dof
    return synth.Arm(types=list(a.type[:n]), lens=list(a.len_vox[:n]), lo_cdeg=list(a.lo_cdeg[:n]),
                     hi_cdeg=list(a.hi_cdeg[:n]), step_cdeg=a.step_cdeg, base=tuple(a.base), samples=a.samples,
                     az0_cdeg=a.az0_cdeg, el0_cdeg=a.el0_cdeg)


def test_tick_grid_matches_oracle_raster(solver):
    dyn = serve.make_dyn_scene(11, 64, column=10)
    scene = solver.scene(dyn.static, ticks=3)
    assert np.array_equal(solver.debug_raster(scene), oracle.raster(dyn.static))
    for t in range(6):
        if t:
            dyn.movers.step(64)
        boxes = dyn.movers.boxes()
        if t == 5:
            boxes = np.concatenate([boxes] * 5)   # more boxes than one launch takes
        say("tick", t, "moving boxes", len(boxes))
        solver.set_dynamic(scene, boxes, t)
        assert np.array_equal(solver.debug_raster(scene), oracle.raster(dyn.at(boxes))), t
    # a scene without room for grids of ticks
    static = solver.scene(dyn.static)
    with pytest.raises(msc.MscError) as e:
        solver.set_dynamic(static, boxes, 0)
    assert e.value.status == msc.E_NOMEM


def test_served_requests_and_replans_match_oracle(solver):
    solver.set_lanes(4)
    try:
        loop = serve.ServingLoop(solver, nscenes=3, seed=2, rate=150.0, keep_log=True, templates=60, n=64,
                                 dof_range=(4, 5), w_range=(4, 10), arm_for=small_arm, ticks_per_waypoint=2,
                                 tick_grids=16)
        rep = loop.run(seconds=1.0, warmup_s=0.0)
        say("serve summary", rep.summary())
        assert rep.served > 40 and rep.unserved == 0
        kinds = {}
        for i, (kind, si, tick, st, res, spec) in enumerate(rep.done_log):
            occ = oracle.raster(loop.scene_at(si, tick))
            arm = spec_arm(spec)
            target = tuple(spec.c.target)
            if kind == "reach":
                r = oracle.reach(arm, occ, target, keep_sets=False)
                ost, ores = r.status, r.pose
            else:
                start = np.asarray(spec.start) // spec.step
                ost, ores, _ = oracle.plan_path(arm, occ, start, target, spec.waypoints, 1)
            assert st == ost, (kind, i, tick, st, ost, spec.error)
            if st == msc.OK:
                assert np.array_equal(res, ores), (kind, i, tick)
            kinds[kind] = kinds.get(kind, 0) + 1
            if i < 8:
                # the same query alone, on a scene holding only this tick's grid
                alone = solver.scene(loop.scene_at(si, tick))
                if kind == "reach":
                    ast, ares = solver.reach(alone, arm, target)
                else:
                    ast, ares = solver.path(alone, arm, start, target, spec.waypoints, 1)
                assert ast == st and (st != msc.OK or np.array_equal(ares, res)), (kind, i)
        say("checked against the oracle:", kinds, "replans:", len(rep.replan_log))
        assert kinds.get("reach", 0) > 10 and kinds.get("path", 0) > 3
        for r in rep.replan_log:
            occ = oracle.raster(loop.scene_at(r["scene_idx"], r["tick"]))
            arm = synth.Arm(types=r["arm_types"], lens=r["arm_lens"], lo_cdeg=r["lo_cdeg"], hi_cdeg=r["hi_cdeg"],
                            step_cdeg=r["step"], base=r["base"])
            ost, opath, _ = oracle.replan_path(arm, occ, r["start"], r["target"], r["waypoints"], r["delta"],
                                               r["ref"])
            assert r["status"] == ost, (r["tick"], r["status"], ost, r["error"])
            if ost == msc.OK:
                assert np.array_equal(r["path"], opath)
    finally:
        solver.set_lanes(0)


def test_forced_replan(solver):
    """A path executing on the server, a one-voxel box placed at a joint of a later
    waypoint (dilated by 2, away from the current pose): the server's step replans the
    rest of the path from the current pose; the new path starts there, every row is
    clear on the oracle's raster of that tick, and it ends on the target."""
    arm = synth.arm_c2()
    solver.set_lanes(2)
    try:
        for seed in range(3, 14):
            dyn = serve.make_dyn_scene(seed)
            scene = solver.scene(dyn.static, ticks=2)
            occ0 = oracle.raster(dyn.static)
            pf = lambda qq: oracle.poses(arm, occ0, qq)  # noqa: E731
            start, _, _ = synth.first_valid_pose(synth.rng_for(8, seed), arm, pf)
            _, target = synth.walk_target(synth.rng_for(8, seed, 1), arm, start, 16, 1, pf)
            solver.server_start()
            try:
                solver.set_dynamic(scene, np.zeros((0, 6), np.int32), 0)
                solver.server_step(0)
                spec = msc.QuerySpec(scene, arm, target, start=start, waypoints=16, delta=1, execute_ticks=8)
                st, path, _ = solver.wait(solver.submit(spec))
                if st != msc.OK:
                    continue
                _, j0 = oracle.pose_joints(arm, occ0, path[0])
                best, where = 0.0, None
                for w in range(2, 16):
                    _, jw = oracle.pose_joints(arm, occ0, path[w])
                    for p in jw[1:]:
                        dmin = np.sqrt(((j0 - p) ** 2).sum(axis=1)).min()
                        if dmin > best:
                            best, where = dmin, p
                if best <= 4.0:
                    continue
                box = np.array([[where[0], where[1], where[2], 1, 1, 1]], np.int32)
                solver.set_dynamic(scene, box, 1)
                rep = solver.server_step(1)
                say("seed", seed, "step report", rep)
                if rep["replans"] == 0:
                    continue   # the voxel also hit the current pose
                got, t0 = [], time.time()
                while not got and time.time() - t0 < 30.0:
                    got = solver.take_replans()
                    time.sleep(0.001)
                assert len(got) == 1
                r = got[0]
                assert r["tick"] == 1 and r["depth"] == 1 and np.array_equal(r["start"], path[0])
                assert np.array_equal(r["ref"], path)
                occ1 = oracle.raster(dyn.at(box))
                if r["status"] == msc.OK:
                    valid, ends = oracle.poses(arm, occ1, r["path"])
                    assert valid.all() and tuple(ends[-1]) == tuple(int(v) for v in target)
                    assert np.array_equal(r["path"][0], path[0])
                    assert np.abs(np.diff(r["path"], axis=0)).max() <= 1
                else:
                    assert r["status"] in (msc.NO_REACH, msc.NO_PATH)
                # the replan executes in place of the old path
                assert solver.server_step(2)["executing"] == (1 if r["status"] == msc.OK else 0)
                return
            finally:
                solver.server_stop()
        pytest.fail("no seed produced a replan")
    finally:
        solver.set_lanes(0)


def test_tickets_and_error_messages(solver):
    arm = small_arm(4)
    dyn = serve.make_dyn_scene(3, 64, column=10)
    scene = solver.scene(dyn.static)
    occ = oracle.raster(dyn.static)
    _, end, _ = synth.first_valid_pose(synth.rng_for(9, 0), arm, lambda q: oracle.poses(arm, occ, q))
    solver.set_lanes(1)
    solver.server_start()
    try:
        d = ctypes.c_int32()
        assert solver.lib.msc_server_poll(solver.ctx, 987654, ctypes.byref(d)) == msc.E_STATE
        assert solver.lib.msc_server_wait(solver.ctx, 987654) == msc.E_STATE
        spec = msc.QuerySpec(scene, arm, end)
        t = solver.submit(spec)
        st, pose, _ = solver.wait(t)
        r = oracle.reach(arm, occ, end, keep_sets=False)
        assert st == r.status == msc.OK and np.array_equal(pose, r.pose)
        # reported once
        assert solver.lib.msc_server_wait(solver.ctx, t) == msc.E_STATE
        assert solver.lib.msc_server_poll(solver.ctx, t, ctypes.byref(d)) == msc.E_STATE
        bad = msc.QuerySpec(scene, arm, (64, 0, 0))
        st, _, _ = solver.wait(solver.submit(bad))
        assert st == msc.E_ARG and "target outside the grid" in bad.error
    finally:
        solver.server_stop()
        solver.set_lanes(0)


def test_admission_by_queue_depth(solver):
    """With a queue limit the server refuses submissions (E_CAPACITY, no ticket) while that
    many wait for a lane; every admitted query completes with the answer it has alone
    (the parity tests tie those to the oracle), and a refused one can be submitted again.
    Eight-DOF path queries on one lane keep the queue full while the submissions arrive."""
    qs = [synth.query_c2(seed, solver.pose_fn_for) for seed in range(4)]
    scenes = [solver.scene(q.scene) for q in qs]
    alone = [solver.path(sc, q.arm, q.start, q.target, q.waypoints, q.max_delta) for sc, q in zip(scenes, qs)]
    solver.set_lanes(1)
    solver.server_start()
    try:
        solver.server_set_limit(1)
        admitted, refused = [], []
        for k in range(16):
            i = k % len(qs)
            q = qs[i]
            spec = msc.QuerySpec(scenes[i], q.arm, q.target, start=q.start, waypoints=q.waypoints, delta=q.max_delta)
            ticket = solver.submit(spec, shed=True)
            (refused if ticket is None else admitted).append((ticket, spec, i))
        say("admitted", len(admitted), "refused", len(refused))
        assert admitted and refused
        for ticket, spec, i in admitted:
            st, path, _ = solver.wait(ticket)
            assert st == alone[i][0]
            if st == msc.OK:
                assert np.array_equal(path, alone[i][1])
        _, spec, i = refused[0]
        st, path, _ = solver.wait(solver.submit(spec))
        assert st == alone[i][0]
        assert solver.lib.msc_server_set_limit(solver.ctx, -1) == msc.E_ARG
        solver.server_set_limit(0)
    finally:
        solver.server_stop()
        solver.set_lanes(0)
