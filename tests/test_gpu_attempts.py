"""GPU parity of the path's attempt order when attempts run together.

When the first tube search of a path query fails, the library searches the remaining
(reach pose, tube radius) attempts in groups, one launch per group and one block per
attempt.  The answer, the reach pose and radius that gave it, and the number of attempts
up to it in search order (for each reach pose, each radius in turn: "Filtering for
smoothness"; another reach pose, Step 3 of "The procedure for IK solution") must be the
oracle's, attempt by attempt; replanning ("Dynamic Obstacles") takes every pose's first
radius with a path and keeps the path nearest the original one."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc

from cases import tiny_case
from test_oracle_order import retry_case


def say(*a):
    print(*a, flush=True)


def one_at_a_time(arm, occ, start, target, W, r0, r1, retries):
    """Every attempt in search order with the oracle's tube search: (reach result,
    [(pose, radius, path or None)])."""
    lim_lo, lim_hi = oracle.arm_limits(arm)
    wlo = np.maximum(lim_lo, start - W)
    whi = np.minimum(lim_hi, start + W)
    res = oracle.reach(arm, occ, target, want=retries, lo=wlo, hi=whi, ref=start, keep_sets=False)
    tries = []
    if res.status == oracle.OK:
        radii = [r0] if r1 == r0 else [r0, r1]
        for i, q in enumerate(res.sols):
            for r in radii:
                tries.append((i, r, oracle.tube_search(arm, occ, start, np.asarray(q, np.int64), W, 1, r,
                                                       lim_lo, lim_hi)))
    return res, tries


SEEDS = list(range(24))


def retry_scene(seed):
    """The scene of retry_case(seed)."""
    return tiny_case(2000 + seed, 4, 3000, nbox=8, n=22, nsph=3)[1]


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS)
def test_first_path_in_search_order(solver, seed):
    arm, occ, start, target, W = retry_case(seed)
    scene = solver.scene(retry_scene(seed))
    # PROFILE times every launch of the groups of attempts
    for r0, r1, retries, flags in ((0, 1, 4, 0), (0, 1, 4, msc.PROFILE), (0, 0, 6, 0), (0, 2, 8, 0)):
        say("attempts", seed, r0, r1, retries, flags)
        res, tries = one_at_a_time(arm, occ, start, target, W, r0, r1, retries)
        st, path = solver.path(scene, arm, start, target, W, 1, tube_r0=r0, tube_r1=r1, retries=retries,
                               flags=flags)
        if res.status != oracle.OK:
            assert st == msc.NO_REACH
            continue
        first = next((k for k, t in enumerate(tries) if t[2] is not None), None)
        s = solver.stats()
        if first is None:
            assert st == msc.NO_PATH
            assert s["attempts"] == len(tries)
        else:
            i, r, p = tries[first]
            assert st == msc.OK
            assert np.array_equal(path, p)
            assert (s["reach_index"], s["tube_r"], s["attempts"]) == (i, r, first + 1)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", SEEDS[:12])
def test_replan_over_every_pose(solver, seed):
    arm, occ, start, target, W = retry_case(seed)
    scene = solver.scene(retry_scene(seed))
    # the original path: the start pose held (every candidate differs from it)
    ref = np.repeat(np.asarray(start, np.int64)[None, :], W + 1, axis=0)
    for r0, r1, retries in ((0, 1, 4), (0, 1, 8)):
        say("replan attempts", seed, r0, r1, retries)
        st, path = solver.replan(scene, arm, start, target, W, 1, ref, tube_r0=r0, tube_r1=r1, retries=retries)
        rst, rpath, _ = oracle.replan_path(arm, occ, start, target, W, 1, ref, r0=r0, r1=r1, retries=retries)
        assert st == rst
        if st == msc.OK:
            assert np.array_equal(path, rpath)


def test_cases_exercise_later_attempts():
    """Several of the cases above find their path only after the first attempt, or none."""
    later = 0
    for seed in SEEDS[:12]:
        arm, occ, start, target, W = retry_case(seed)
        res, tries = one_at_a_time(arm, occ, start, target, W, 0, 1, 4)
        if res.status == oracle.OK and (tries[0][2] is None):
            later += 1
    assert later >= 3, later


@pytest.mark.gpu
@pytest.mark.parametrize("lanes", [0, 3])
def test_batched_attempts(solver, lanes):
    """The same order on worker lanes (no more attempts than the order can need) and on
    the control lane of a batch (every attempt after a failed first one)."""
    say("batched attempts, lanes", lanes)
    cases = [retry_case(seed) for seed in SEEDS]
    specs = [msc.QuerySpec(solver.scene(retry_scene(seed)), arm, target, start=start, waypoints=W, delta=1)
             for seed, (arm, occ, start, target, W) in zip(SEEDS, cases)]
    solver.set_lanes(lanes)
    try:
        got = solver.batch(specs, tube_r0=0, tube_r1=1, retries=4)
    finally:
        solver.set_lanes(0)
    for (arm, occ, start, target, W), (st, path, _lat) in zip(cases, got):
        rst, rpath, _ = oracle.plan_path(arm, occ, start, target, W, 1, r0=0, r1=1, retries=4)
        assert st == rst
        if st == msc.OK:
            assert np.array_equal(path, rpath)
