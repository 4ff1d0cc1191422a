"""GPU parity of midcourse replanning (msc_replan: the candidate path nearest the
original one) with the oracle, through the C ABI: tiny chains with random reference
paths, a reference equal to the first path (msc_path's answer comes back), and
full-size 8-DOF queries with a straight reference toward a drawn pose."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc, synth

from test_gpu_parity import say
from test_oracle_replan import path_case


def reference(rng, start, W, span):
    goal = np.asarray(start, np.int64) + rng.integers(-span, span + 1, size=len(start))
    return np.rint(np.linspace(start, goal, W + 1)).astype(np.int64)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(12))
def test_replan_tiny(solver, seed):
    arm, sc, occ, start, target, W = path_case(seed, with_scene=True)
    scene = solver.scene(sc)
    rng = synth.rng_for(914, seed)
    ref = reference(rng, start, W, 3)
    say("replan tiny", seed)
    st, path = solver.replan(scene, arm, start, target, W, 1, ref)
    rst, rpath, _ = oracle.replan_path(arm, occ, start, target, W, 1, ref)
    assert st == rst
    if st == msc.OK:
        assert np.array_equal(path, rpath)
    st1, p1 = solver.path(scene, arm, start, target, W, 1)
    if st1 == msc.OK:
        st2, p2 = solver.replan(scene, arm, start, target, W, 1, p1)
        assert st2 == msc.OK and np.array_equal(p2, p1)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [0, 3])
def test_replan_full_size(solver, seed):
    q = synth.query_c2(seed, solver.pose_fn_for)
    scene = solver.scene(q.scene)
    occ = oracle.raster(q.scene)
    rng = synth.rng_for(915, seed)
    ref = reference(rng, q.start, q.waypoints, 16)
    say("replan c2", seed)
    st, path = solver.replan(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta, ref, split_m=6)
    rst, rpath, _ = oracle.replan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, ref, m=6)
    assert st == rst
    if st == msc.OK:
        assert np.array_equal(path, rpath)


@pytest.mark.gpu
def test_batched_replans_equal_alone(solver):
    """Queries that carry an original path, solved by msc_batch over worker lanes, give
    msc_replan's answers."""
    specs, alone = [], []
    for seed in range(8):
        arm, sc, occ, start, target, W = path_case(seed, with_scene=True)
        scene = solver.scene(sc)
        ref = reference(synth.rng_for(917, seed), start, W, 3)
        specs.append(msc.QuerySpec(scene, arm, target, start=start, waypoints=W, delta=1, ref=ref))
        alone.append(solver.replan(scene, arm, start, target, W, 1, ref))
    solver.set_lanes(3)
    try:
        res = solver.batch(specs)
    finally:
        solver.set_lanes(0)
    for (st, path, _), (ast, apath) in zip(res, alone):
        assert st == ast
        if st == msc.OK:
            assert np.array_equal(path, apath)


@pytest.mark.gpu
def test_replan_argument_errors(solver):
    arm, sc, occ, start, target, W = path_case(0, with_scene=True)
    scene = solver.scene(sc)
    ref = np.repeat(np.asarray(start, np.int64)[None, :], W + 1, axis=0)
    a = msc.make_arm(arm)
    s = np.ascontiguousarray(np.asarray(start, np.int32) * a.step_cdeg)
    t = np.ascontiguousarray(np.asarray(target, np.int32))
    out = np.zeros((W + 1) * a.dof, np.int32)
    bad = np.ascontiguousarray(ref.astype(np.int32) * a.step_cdeg + 1)   # not a multiple of the step
    o = msc.make_opts()

    def P(x):
        return x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))

    rc = solver.lib.msc_replan(solver.ctx, scene.handle, ctypes.byref(a), P(s), P(t), W, a.step_cdeg, P(bad),
                               ctypes.byref(o), P(out))
    assert rc == msc.E_ARG
    rc = solver.lib.msc_replan(solver.ctx, scene.handle, ctypes.byref(a), P(s), P(t), W, a.step_cdeg, None,
                               ctypes.byref(o), P(out))
    assert rc == msc.E_ARG
    # a valid call still works after the rejected ones
    st, _ = solver.replan(scene, arm, start, target, W, 1, ref)
    assert st in (msc.OK, msc.NO_REACH, msc.NO_PATH)
