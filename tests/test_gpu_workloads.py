"""Batched workloads against the oracle: shrunken variants of the batched-reach
(128/256^3, DOF 5-8, unwindowed) and batched-path (512^3, 2.5 deg) workloads, built by
the same generators with smaller grids / DOF / steps, solved by msc_batch over worker
lanes and compared bit for bit with the oracle; full-size batched reach queries are
checked by properties (forward-kinematics replay of every returned pose)."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def specs_for(solver, qs):
    scenes, specs = {}, []
    for q in qs:
        key = id(q.scene)
        if key not in scenes:
            scenes[key] = solver.scene(q.scene)
        sc = scenes[key]
        if q.start is None:
            specs.append(msc.QuerySpec(sc, q.arm, q.target))
        else:
            specs.append(msc.QuerySpec(sc, q.arm, q.target, start=q.start, waypoints=q.waypoints, delta=q.max_delta))
    return specs


@pytest.mark.parametrize("n,max_dof", [(64, 6), (128, 5)])
def test_c3_shrunken_batch_vs_oracle(solver, n, max_dof):
    qs = synth.queries_c3(oracle.pose_fn_for, scenes=3, per_scene=4, n=n, max_dof=max_dof)
    solver.set_lanes(4)
    try:
        res = solver.batch(specs_for(solver, qs))
    finally:
        solver.set_lanes(0)
    for q, (st, pose, _) in zip(qs, res):
        occ = oracle.raster(q.scene)
        ref = oracle.reach(q.arm, occ, q.target, m=(q.arm.dof + 1) // 2 + 1, keep_sets=False)
        say("c3", n, q.arm.dof, st, ref.status)
        assert st == ref.status
        if st == msc.OK:
            assert np.array_equal(pose, ref.pose)


def test_c4_shrunken_batch_vs_oracle(solver):
    qs = synth.queries_c4(oracle.pose_fn_for, scenes=2, per_scene=4, n=96, step_cdeg=1000, w_range=(4, 8), dof=6,
                          lens_scale=1.0)
    solver.set_lanes(3)
    try:
        res = solver.batch(specs_for(solver, qs))
    finally:
        solver.set_lanes(0)
    for q, (st, path, _) in zip(qs, res):
        occ = oracle.raster(q.scene)
        rst, rpath, _ = oracle.plan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, m=3)
        say("c4", q.waypoints, st, rst)
        assert st == rst
        if st == msc.OK:
            assert np.array_equal(path, rpath)


def test_c3_full_size_properties(solver):
    """Full-size scenes and 8-DOF arms, unwindowed joints: every returned pose replays
    clear onto its target (checked with the oracle's replay); NO_REACH is allowed."""
    qs = synth.queries_c3(solver.pose_fn_for, scenes=2, per_scene=4)
    solver.set_lanes(4)
    try:
        res = solver.batch(specs_for(solver, qs))
    finally:
        solver.set_lanes(0)
    ok = 0
    for q, (st, pose, lat) in zip(qs, res):
        say("c3 full", q.scene.n, q.arm.dof, st, "%.1f ms" % lat)
        assert st in (msc.OK, msc.NO_REACH)
        if st == msc.OK:
            valid, ends = oracle.poses(q.arm, oracle.raster(q.scene), pose[None, :])
            assert valid[0] and tuple(ends[0]) == tuple(q.target)
            ok += 1
    assert ok > 0
