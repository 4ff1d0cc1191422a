"""Pins of the oracle of the paper's gap search ("Discretization of the segment
articulations", "The gap in gMS", "Exact IK solution with discretized segment mappings").

* The quiver against its closed form: ring counts, unit vectors, the poles and the
  equator, mirror symmetry of every ring, near-constant density away from the poles,
  and the ~10^4 vectors of a 2 degree quiver the paper's thread count implies.
* The pruned search (eqs 5-8) against the unpruned enumeration of every (i, j, l): the
  pruning loses no solution; the array form against the one-at-a-time form.
* A constructed case: the straight vertical arm reaches the point above the base at its
  full length, its free vector exactly L3.
* Every solution replayed: end point, gap length within eps, flexion limits; the exact
  end point of the 8-DOF text closes on the target.
"""
import math

import numpy as np
import pytest

from oracle import gms
from paper_1906_10678_amd import synth

from cases import tiny_scene


@pytest.mark.parametrize("step", [3000, 2000, 1500, 1000, 500, 200])
def test_quiver_rings_follow_the_closed_form(step):
    D = step / 100.0
    n = 36000 // step
    counts = gms.ring_counts(step)
    assert len(counts) == 180 // D + 1
    assert counts[0] == counts[-1] == 1
    for i, m in enumerate(counts[1:-1], start=1):
        e = -90 + i * D
        want = n * math.cos(math.radians(e))
        assert m >= 4 and (m == 4 or abs(m - want) <= 0.5 + 1e-9)
    Q = gms.quiver(step)
    assert len(Q) == sum(counts)
    assert np.allclose(np.linalg.norm(Q, axis=1), 1.0, atol=1e-15)
    assert np.allclose(Q[0], [0, 0, -1], atol=1e-16) and np.allclose(Q[-1], [0, 0, 1], atol=1e-16)
    if 9000 % step == 0:
        # the equator ring keeps every azimuth: z == 0 exactly, azimuth j * D
        i0 = 9000 // step
        assert counts[i0] == n
        off = sum(counts[:i0])
        eq = Q[off:off + n]
        assert (eq[:, 2] == 0.0).all()
        az = np.degrees(np.arctan2(eq[:, 1], eq[:, 0])) % 360
        assert np.allclose(az, np.arange(n) * D, atol=1e-9)


def test_quiver_rings_are_mirror_symmetric_and_nearly_uniform():
    step = 500
    Q = gms.quiver(step)
    counts = gms.ring_counts(step)
    start = 0
    for i, m in enumerate(counts):
        ring = Q[start:start + m]
        start += m
        mirrored = ring * np.array([1, -1, 1])
        for v in mirrored:
            assert np.min(np.abs(ring - v).sum(axis=1)) < 1e-12
        e = -90 + i * step / 100.0
        if m > 4:
            spacing = 360.0 / m * math.cos(math.radians(e))   # great-circle spacing along the ring
            assert 0.9 * step / 100.0 <= spacing <= 1.1 * step / 100.0


def test_two_degree_quiver_has_about_ten_thousand_vectors():
    # the paper's GPU kernel runs one thread per segment-2 vector: about 10^4 at 2 degrees
    n = len(gms.quiver(200))
    assert 10000 <= n <= 10600


def tiny_gms(seed, step=3000, n=20, nbox=3):
    rng = synth.rng_for(970, seed)
    lens = rng.uniform(2.5, 5.0, size=4)
    arm = gms.GmsArm(lens, (n // 2, n // 2, 1), step_cdeg=step, samples=6, seg1_min_el_cdeg=0,
                     max_flex_cdeg=(12000, 13500, 13500), eps=0.6)
    scene = tiny_scene(rng, n, nbox, 0, 1, base=arm.base, column=4)
    return arm, scene, rng


def targets_of(arm, occ, rng, count):
    """Targets near the end of random chains of quiver vectors (free voxels)."""
    Q = gms.quiver(arm.step_cdeg)
    out = []
    for _ in range(count * 20):
        idx = rng.integers(0, len(Q), size=4)
        p = np.array(arm.base, float)
        for k in range(4):
            p = p + arm.lens[k] * Q[idx[k]]
        v = np.array([gms.round_half_away(c) for c in p])
        if (v >= 0).all() and (v < occ.shape[0]).all() and occ[v[2], v[1], v[0]] == 0:
            out.append(v)
        if len(out) == count:
            break
    return out


@pytest.mark.parametrize("seed", range(4))
def test_pruning_loses_no_solution(seed):
    arm, scene, rng = tiny_gms(seed)
    import oracle
    occ = oracle.raster(scene)
    found = 0
    for t in targets_of(arm, occ, rng, 3):
        a = gms.solutions_plain(arm, occ, t, prune=True)
        b = gms.solutions_plain(arm, occ, t, prune=False)
        assert a == b
        assert gms.solutions(arm, occ, t) == a
        found += len(a)
    assert found > 0


def test_array_form_equals_one_at_a_time_on_a_larger_quiver():
    import oracle
    arm, scene, rng = tiny_gms(9, step=2000, n=24, nbox=4)
    occ = oracle.raster(scene)
    for t in targets_of(arm, occ, rng, 2):
        assert gms.solutions(arm, occ, t) == gms.solutions_plain(arm, occ, t)


def test_straight_arm_reaches_straight_up():
    L = [3.0, 4.0, 5.0, 2.0]
    arm = gms.GmsArm(L, (8, 8, 0), step_cdeg=3000, samples=4, eps=1e-6)
    occ = np.zeros((20, 20, 20), np.uint8)
    t = (8, 8, int(sum(L)))
    sols = gms.solutions_plain(arm, occ, t)
    top = len(gms.quiver(3000)) - 1                      # the +z pole
    assert (top, top, top) in sols
    v = gms.vectors(arm, t, (top, top, top))
    assert np.allclose(v[2], [0, 0, 5.0], atol=1e-12)   # the free vector spans exactly L3


@pytest.mark.parametrize("seed", range(3))
def test_solutions_replay_and_exact_end_point(seed):
    import oracle
    arm, scene, rng = tiny_gms(seed + 20)
    occ = oracle.raster(scene)
    Q = gms.quiver(arm.step_cdeg)
    for t in targets_of(arm, occ, rng, 2):
        for sol in gms.solutions(arm, occ, t)[:20]:
            v = gms.vectors(arm, t, sol)
            s1, s2, v3, s4, s3, s4e = v
            end = np.array(arm.base, float) + s1 + s2 + v3 + s4
            assert np.allclose(end, t, atol=1e-9)
            assert abs(np.linalg.norm(v3) - arm.lens[2]) <= arm.eps
            assert abs(np.linalg.norm(s3) - arm.lens[2]) <= 1e-9
            assert np.allclose(np.array(arm.base, float) + s1 + s2 + s3 + s4e, t, atol=1e-9)
            units = [Q[sol[0]], Q[sol[1]], v3 / np.linalg.norm(v3), Q[sol[2]]]
            for k in range(3):
                ang = math.degrees(math.acos(max(-1.0, min(1.0, float(units[k] @ units[k + 1])))))
                assert ang <= arm.max_flex_cdeg[k] / 100.0 + 1e-6
            assert Q[sol[0]][2] >= -1e-9                 # segment 1 in the upper hemisphere
