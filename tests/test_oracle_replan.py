"""Pins of the oracle's replanning objective ("Dynamic Obstacles": of the candidate
paths, the one with the least mean distance to the original path).  The candidates are
the paths of the first reach poses in the canonical order; the checks: the original
path itself is chosen back, the chosen path is no farther from the reference than any
candidate (enumerated one by one), a reference equal to a later candidate selects it,
and every chosen path is a valid path (FK replay, moves of at most delta)."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import synth

from cases import tiny_case


def path_case(seed, with_scene=False):
    arm, sc, rng = tiny_case(seed, 4, 3000, n=24, nbox=4)
    occ = oracle.raster(sc)
    pf = oracle.pose_fn_for(arm, sc)
    start, _, _ = synth.first_valid_pose(rng, arm, pf, batch=256)
    W = 6
    _, end = synth.walk_target(rng, arm, start, W, 1, pf)
    if with_scene:
        return arm, sc, occ, start, tuple(int(v) for v in end), W
    return arm, occ, start, tuple(int(v) for v in end), W


def candidates(arm, occ, start, target, W, retries=4):
    lim_lo, lim_hi = oracle.arm_limits(arm)
    wlo = np.maximum(lim_lo, start - W)
    whi = np.minimum(lim_hi, start + W)
    res = oracle.reach(arm, occ, target, want=retries, lo=wlo, hi=whi, ref=start, keep_sets=False)
    out = []
    for q in res.sols:
        for r in (1, 2):
            p = oracle.tube_search(arm, occ, np.asarray(start, np.int64), q, W, 1, r, lim_lo, lim_hi)
            if p is not None:
                out.append(np.asarray(p, np.int64))
                break
    return out


def check_valid(arm, occ, path, start, target):
    assert np.array_equal(path[0], start)
    assert np.abs(np.diff(path, axis=0)).max() <= 1
    valid, ends = oracle.poses(arm, occ, np.asarray(path, np.int32))
    assert valid.all()
    assert tuple(ends[-1]) == tuple(target)


@pytest.mark.parametrize("seed", range(12))
def test_original_path_is_chosen_back(seed):
    arm, occ, start, target, W = path_case(seed)
    st, path, _ = oracle.plan_path(arm, occ, start, target, W, 1)
    if st != oracle.OK:
        pytest.skip("no path for this draw")
    st2, again, _ = oracle.replan_path(arm, occ, start, target, W, 1, path)
    assert st2 == oracle.OK
    assert np.array_equal(again, path)


@pytest.mark.parametrize("seed", range(12))
def test_choice_is_the_nearest_candidate(seed):
    arm, occ, start, target, W = path_case(seed)
    cands = candidates(arm, occ, start, target, W)
    if not cands:
        pytest.skip("no path for this draw")
    rng = synth.rng_for(913, seed)
    ref = np.asarray(start, np.int64)[None, :] + rng.integers(-2, 3, size=(W + 1, arm.dof))
    st, path, _ = oracle.replan_path(arm, occ, start, target, W, 1, ref)
    assert st == oracle.OK
    cost = np.abs(np.asarray(path, np.int64) - ref).sum()
    costs = [np.abs(c - ref).sum() for c in cands]
    assert cost == min(costs)
    # ties go to the earliest candidate
    assert np.array_equal(path, cands[int(np.argmin(costs))])
    check_valid(arm, occ, np.asarray(path), start, target)


@pytest.mark.parametrize("seed", range(12))
def test_reference_equal_to_a_later_candidate_selects_it(seed):
    arm, occ, start, target, W = path_case(seed)
    cands = candidates(arm, occ, start, target, W)
    later = [c for c in cands[1:] if not np.array_equal(c, cands[0])]
    if not later:
        pytest.skip("fewer than two distinct candidate paths")
    st, path, _ = oracle.replan_path(arm, occ, start, target, W, 1, later[-1])
    assert st == oracle.OK
    assert np.array_equal(path, later[-1])
