"""Pins of the oracle's path search.

Reading of "Smooth sequence computation" and "Filtering for smoothness": the path
is worked backward from the reach pose; each waypoint pose must be clear of
obstacles and within a bounded joint change of its neighbour, and among the
candidates the one closest in configuration is taken.  Concretely: poses at
waypoint w lie in a tube of radius r around the integer guide from the start to the
reach pose, every move changes each joint by at most delta, and the backward choice
is the L1-closest pose to the guide, ties broken by joint values.  The tube radius
is relaxed only after a failure (adaptive relaxation, "Filtering for smoothness").
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import synth

from cases import tiny_case


def round_half_away(fr: Fraction) -> int:
    s = 1 if fr >= 0 else -1
    a = abs(fr)
    fl = a.numerator // a.denominator
    return s * (fl + (1 if a - fl >= Fraction(1, 2) else 0))


@pytest.mark.parametrize("W", [1, 2, 3, 5, 16, 33])
def test_guide_is_rounded_linear_interpolation(W):
    rng = np.random.default_rng(W)
    start = rng.integers(-30, 30, size=8)
    goal = start + rng.integers(-W, W + 1, size=8)
    g = oracle.guide(start, goal, W)
    for w in range(W + 1):
        for k in range(8):
            expect = start[k] + round_half_away(Fraction(int(w * (goal[k] - start[k])), W))
            assert g[w, k] == expect
    assert np.array_equal(g[0], start) and np.array_equal(g[W], goal)
    # |goal - start| <= W  =>  consecutive guide poses differ by at most one step
    assert np.abs(np.diff(g, axis=0)).max() <= 1


def brute_tube(arm, occ, start, goal, W, delta, r, lo, hi):
    """The same search by plain set recursion over explicit pose lists."""
    g = oracle.guide(start, goal, W)
    sets = []
    for w in range(W + 1):
        if w == 0:
            cand = [tuple(start)]
        elif w == W:
            cand = [tuple(goal)]
        else:
            rngs = [range(max(g[w][k] - r, lo[k]), min(g[w][k] + r, hi[k]) + 1) for k in range(len(start))]
            cand = list(itertools.product(*rngs))
        valid, _ = oracle.poses(arm, occ, np.array(cand, np.int32))
        keep = []
        for c, v in zip(cand, valid):
            if not v:
                continue
            if w > 0 and not any(max(abs(a - b) for a, b in zip(c, p)) <= delta for p in sets[-1]):
                continue
            keep.append(c)
        sets.append(keep)
    if tuple(goal) not in sets[W]:
        return None
    path = [tuple(goal)]
    for w in range(W, 0, -1):
        q = path[-1]
        cands = [p for p in sets[w - 1] if max(abs(a - b) for a, b in zip(p, q)) <= delta]
        best = min(cands, key=lambda p: (sum(abs(a - b) for a, b in zip(p, g[w - 1])), p))
        path.append(best)
    return np.array(path[::-1], np.int32)


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("r", [1, 2])
def test_tube_search_matches_brute_force(seed, r):
    arm, scene, rng = tiny_case(seed, 3, 3000, nbox=4)
    occ = oracle.raster(scene)
    lo, hi = oracle.arm_limits(arm)
    q = synth.candidate_poses(rng, arm, 512)
    valid, _ = oracle.poses(arm, occ, q)
    good = q[valid]
    if len(good) < 2:
        pytest.skip("no valid poses drawn")
    start, goal = good[0].astype(np.int64), good[1].astype(np.int64)
    W = int(np.abs(goal - start).max()) + int(rng.integers(0, 3))
    W = max(W, 1)
    a = oracle.tube_search(arm, occ, start, goal, W, 1, r, lo, hi)
    b = brute_tube(arm, occ, start, goal, W, 1, r, lo, hi)
    assert (a is None) == (b is None)
    if a is not None:
        assert np.array_equal(a, b)


def check_path(arm, occ, start, target, W, delta, path):
    assert path.shape == (W + 1, len(start))
    assert np.array_equal(path[0], start)
    assert np.abs(np.diff(path.astype(np.int64), axis=0)).max(initial=0) <= delta
    valid, ends = oracle.poses(arm, occ, path)
    assert valid.all()
    assert tuple(ends[-1]) == tuple(target)
    lo, hi = oracle.arm_limits(arm)
    assert (path >= lo).all() and (path <= hi).all()


@pytest.mark.parametrize("seed", range(8))
def test_plan_path_on_feasible_walks(seed):
    """Targets at the end of a feasible walk of W moves always yield a path whose
    every row is valid, whose moves are within delta and whose end is on the target."""
    arm, scene, rng = tiny_case(seed, 4, 3000, nbox=4, n=24)
    occ = oracle.raster(scene)
    pf = oracle.pose_fn_for(arm, scene)
    start, _, _ = synth.first_valid_pose(rng, arm, pf, batch=256)
    W = int(rng.integers(2, 6))
    _, target = synth.walk_target(rng, arm, start, W, 1, pf)
    st, path, res = oracle.plan_path(arm, occ, start, target, W, 1)
    assert st in (oracle.OK, oracle.NO_PATH)
    assert res.status == oracle.OK  # the walk end is reachable inside the window
    if st == oracle.OK:
        check_path(arm, occ, start, target, W, 1, path)
        # the last row is one of the enumerated reach poses
        assert any(np.array_equal(path[-1], s) for s in res.sols)


def test_invalid_start_is_rejected():
    arm, scene, rng = tiny_case(0, 3, 3000)
    occ = oracle.raster(scene)
    bad = np.array(arm.base)
    occ2 = occ.copy()
    occ2[bad[2], bad[1], bad[0]] = 1
    st, _, _ = oracle.plan_path(arm, occ2, np.zeros(3, np.int64), (1, 1, 1), 3, 1)
    assert st == oracle.E_ARG
    lo, hi = oracle.arm_limits(arm)
    st, _, _ = oracle.plan_path(arm, occ, hi + 1, (1, 1, 1), 3, 1)
    assert st == oracle.E_ARG


def test_zero_waypoints():
    arm, scene, rng = tiny_case(2, 3, 3000)
    occ = oracle.raster(scene)
    pf = oracle.pose_fn_for(arm, scene)
    start, end, _ = synth.first_valid_pose(rng, arm, pf, batch=256)
    st, path, _ = oracle.plan_path(arm, occ, start, end, 0, 1)
    assert st == oracle.OK and np.array_equal(path, start[None, :])
