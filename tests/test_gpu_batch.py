"""Batched execution and the server: every query's result equals the same query solved
alone with msc_reach / msc_path (which the parity suite ties to the oracle), whatever
the lane count and whatever runs beside it."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc, synth

from cases import tiny_case

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def mixed_queries(solver):
    """Reach and path queries over several scenes: C1 seeds, tiny arms, C2 seeds."""
    specs, alone = [], []
    for seed in range(3):
        q = synth.query_c1(seed, oracle.pose_fn_for)
        sc = solver.scene(q.scene)
        specs.append(msc.QuerySpec(sc, q.arm, q.target))
        alone.append(("reach", sc, q.arm, q.target))
    for seed in range(4):
        arm, scn, rng = tiny_case(seed, 4, 3000, nbox=4, n=24)
        pf = oracle.pose_fn_for(arm, scn)
        start, _, _ = synth.first_valid_pose(rng, arm, pf, batch=256)
        _, target = synth.walk_target(rng, arm, start, 4, 1, pf)
        sc = solver.scene(scn)
        specs.append(msc.QuerySpec(sc, arm, target, start=start, waypoints=4, delta=1))
        alone.append(("path", sc, arm, target, start, 4, 1))
    for seed in range(3):
        q = synth.query_c2(seed, solver.pose_fn_for)
        sc = solver.scene(q.scene)
        specs.append(msc.QuerySpec(sc, q.arm, q.target, start=q.start, waypoints=q.waypoints, delta=q.max_delta))
        alone.append(("path", sc, q.arm, q.target, q.start, q.waypoints, q.max_delta))
    return specs, alone


def solve_alone(solver, a):
    if a[0] == "reach":
        return solver.reach(a[1], a[2], a[3])
    return solver.path(a[1], a[2], a[4], a[3], a[5], a[6])


@pytest.mark.parametrize("lanes", [0, 1, 3, 8])
def test_batch_equals_alone(solver, lanes):
    say("batch lanes", lanes)
    solver.set_lanes(lanes)
    try:
        specs, alone = mixed_queries(solver)
        expect = [solve_alone(solver, a) for a in alone]
        got = solver.batch(specs)
        for (st, res, _lat), (est, eres) in zip(got, expect):
            assert st == est
            if st == msc.OK:
                assert np.array_equal(res, eres)
    finally:
        solver.set_lanes(0)


def test_server_alone_vs_mix(solver):
    """Queries submitted while others are in flight, in a shuffled order, give exactly
    the results they give alone."""
    solver.set_lanes(4)
    try:
        specs, alone = mixed_queries(solver)
        expect = [solve_alone(solver, a) for a in alone]
        solver.server_start()
        try:
            order = np.random.default_rng(5).permutation(len(specs))
            tickets = {}
            for i in order:
                tickets[int(i)] = solver.submit(specs[int(i)])
            for i, t in tickets.items():
                st, res, lat = solver.wait(t)
                est, eres = expect[i]
                assert st == est
                if st == msc.OK:
                    assert np.array_equal(res, eres)
                assert lat >= 0
        finally:
            solver.server_stop()
    finally:
        solver.set_lanes(0)


def test_server_admission_by_memory(solver):
    """A query whose device-memory estimate exceeds a lane window is refused at submit."""
    solver.set_lanes(2)
    try:
        q = synth.query_c2(0, solver.pose_fn_for)
        sc = solver.scene(q.scene)
        big = synth.Arm(types=q.arm.types, lens=[250] * 8, lo_cdeg=q.arm.lo_cdeg, hi_cdeg=q.arm.hi_cdeg,
                        step_cdeg=250, base=q.arm.base)
        spec = msc.QuerySpec(sc, big, q.target, start=np.zeros(8, np.int32), waypoints=64, delta=1)
        assert solver.query_bytes(spec) > solver.lane_bytes()
        solver.server_start()
        try:
            with pytest.raises(msc.MscError) as e:
                solver.submit(spec)
            assert e.value.status == msc.E_NOMEM
            # an ordinary query is still served
            ok = msc.QuerySpec(sc, q.arm, q.target, start=q.start, waypoints=q.waypoints, delta=q.max_delta)
            st, _, _ = solver.wait(solver.submit(ok))
            assert st == msc.OK
        finally:
            solver.server_stop()
    finally:
        solver.set_lanes(0)


def test_server_states(solver):
    solver.set_lanes(0)
    with pytest.raises(msc.MscError) as e:
        solver.server_start()
    assert e.value.status == msc.E_STATE


def test_fresh_scenes_on_worker_lanes(solver):
    """Scenes created just before a batch: the raster runs on the control lane's stream
    without the call waiting for it, and the worker lanes wait for it before they read
    the grid.  Every batched answer equals the answer on the same scene solved alone."""
    solver.set_lanes(8)
    try:
        qs = [synth.query_c2(seed, solver.pose_fn_for) for seed in range(8)]
        for rnd in range(3):
            say("fresh scenes round", rnd)
            specs = []
            for q in qs:
                sc = solver.scene(q.scene)   # rasterised now, not waited for
                specs.append(msc.QuerySpec(sc, q.arm, q.target, start=q.start, waypoints=q.waypoints,
                                           delta=q.max_delta))
            got = solver.batch(specs)
            for (st, res, _lat), spec, q in zip(got, specs, qs):
                est, eres = solver.path(spec.scene, q.arm, q.start, q.target, q.waypoints, q.max_delta)
                assert st == est
                if st == msc.OK:
                    assert np.array_equal(res, eres)
    finally:
        solver.set_lanes(0)
