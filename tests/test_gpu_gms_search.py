"""GPU parity of the paper's gap search (msc_gms_reach) with oracle.gms, through the C
ABI: the solution count, the first solutions in (i, j, l) order (exactly) and their
vectors (FP64, 1e-9), on small quivers in small scenes, a 10 degree quiver on a 64^3
grid with an approach cone, and the 2 degree quiver (about 10^4 vectors, the paper's
setting) on a full-size 256^3 scene, where the oracle computes the first solutions.
Every decision is made in FP64 with the same operations on both sides."""
import numpy as np
import pytest

import oracle
from oracle import gms
from paper_1906_10678_amd import msc, synth

from cases import tiny_scene
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def compare(solver, scene, arm, occ, t, want=16, full=True, first_only=False):
    st, count, sols, vec = solver.gms_reach(scene, arm, t, want, first_only=first_only)
    if full:
        ref = gms.solutions(arm, occ, t)
        if first_only:
            assert min(want, len(ref)) <= count <= len(ref), (count, len(ref))
        else:
            assert count == len(ref), (count, len(ref))
    else:
        ref = gms.solutions(arm, occ, t, limit=want)
        assert count >= len(ref)
    if not ref:
        assert st == msc.NO_REACH
        return 0
    assert st == msc.OK
    k = min(want, len(ref))
    assert [tuple(x) for x in sols[:k]] == ref[:k]
    for m in range(k):
        assert np.allclose(vec[m], gms.vectors(arm, t, ref[m]), atol=1e-9, rtol=0)
    return len(ref)


def small_case(seed, step, n, nbox):
    rng = synth.rng_for(971, seed)
    lens = rng.uniform(2.5, 5.0, size=4)
    arm = gms.GmsArm(lens, (n // 2, n // 2, 1), step_cdeg=step, samples=6, seg1_min_el_cdeg=0,
                     max_flex_cdeg=(12000, 13500, 13500), eps=0.6)
    sc = tiny_scene(rng, n, nbox, 0, 1, base=arm.base, column=4)
    return arm, sc, rng


def targets_of(arm, occ, rng, count):
    Q = gms.quiver(arm.step_cdeg)
    out = []
    for _ in range(count * 30):
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


@pytest.mark.parametrize("step", [3000, 2000, 1500])
def test_gms_small(solver, step):
    total = 0
    for seed in range(4):
        arm, sc, rng = small_case(seed, step, 24, 4)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        for t in targets_of(arm, occ, rng, 3):
            say("gms small", step, seed, tuple(t))
            total += compare(solver, scene, arm, occ, t)
            compare(solver, scene, arm, occ, t, want=4, first_only=True)
    assert total > 0


def test_gms_cone_and_blocked_ends(solver):
    arm, sc, rng = small_case(7, 2000, 24, 3)
    arm.approach = (0, -9000, 6000)         # the last segment within 60 degrees of straight down
    occ = oracle.raster(sc)
    scene = solver.scene(sc)
    for t in targets_of(arm, occ, rng, 4):
        compare(solver, scene, arm, occ, t)
    blocked = np.argwhere(occ)
    if len(blocked):
        z, y, x = blocked[0]
        st, count, sols, _ = solver.gms_reach(scene, arm, (x, y, z), 4)
        assert st == msc.NO_REACH and count == 0


def test_gms_medium_ten_degrees(solver):
    rng = synth.rng_for(972, 0)
    n = 64
    arm = gms.GmsArm([14.0, 12.0, 10.0, 6.0], (32, 32, 0), step_cdeg=1000, samples=8, seg1_min_el_cdeg=0,
                     max_flex_cdeg=(13000, 13000, 13000), approach=(0, -9000, 7000), eps=0.75)
    sc = synth.random_scene(rng, n, 1, 6, (4, 12), 2, (2, 5), base=arm.base, column=16)
    occ = oracle.raster(sc)
    scene = solver.scene(sc)
    total = 0
    for t in targets_of(arm, occ, rng, 3):
        say("gms medium", tuple(t))
        total += compare(solver, scene, arm, occ, t, want=32)
    assert total > 0


def test_gms_two_degrees_full_size(solver):
    """The paper's setting: a 2 degree quiver (about 10^4 vectors) on the 8-DOF workload's
    256^3 scene; the oracle computes the first solutions in order."""
    q = synth.query_c2(0, solver.pose_fn_for)
    occ = oracle.raster(q.scene)
    scene = solver.scene(q.scene)
    arm = gms.GmsArm([60.0, 50.0, 40.0, 25.0], (128, 128, 0), step_cdeg=200, samples=8, seg1_min_el_cdeg=0,
                     max_flex_cdeg=(12000, 12000, 12000), approach=(0, -9000, 4500), eps=0.5)
    say("gms 2 deg", tuple(q.target))
    found = compare(solver, scene, arm, occ, np.asarray(q.target), want=8, full=False)
    assert found > 0


def test_gms_first_solutions_full_size(solver):
    """msc_gms_reach_first on the 2 degree quiver: the first solutions and their vectors
    equal the oracle's and the full search's; the count is at least the number wanted and
    at most the full search's."""
    arm = gms.GmsArm([60.0, 50.0, 40.0, 25.0], (128, 128, 0), step_cdeg=200, samples=8, seg1_min_el_cdeg=0,
                     max_flex_cdeg=(12000, 12000, 12000), approach=(0, -9000, 4500), eps=0.5)
    answered = 0
    for seed in (0, 1, 2, 3):
        q = synth.query_c2(seed, solver.pose_fn_for)
        occ = oracle.raster(q.scene)
        scene = solver.scene(q.scene)
        t = np.asarray(q.target)
        say("gms first", seed, tuple(t))
        st_a, count_a, sols_a, vec_a = solver.gms_reach(scene, arm, t, 8)
        st_f, count_f, sols_f, vec_f = solver.gms_reach(scene, arm, t, 8, first_only=True)
        assert st_f == st_a
        assert np.array_equal(sols_f, sols_a) and np.array_equal(vec_f, vec_a)
        assert min(8, count_a) <= count_f <= count_a
        if st_a == msc.OK:
            answered += 1
            ref = gms.solutions(arm, occ, t, limit=8)
            assert [tuple(x) for x in sols_f] == ref[:len(sols_f)]
    assert answered >= 2


def test_gms_argument_errors(solver):
    """Bad arguments are rejected before any GPU work, with E_ARG."""
    arm, sc, rng = small_case(0, 3000, 24, 2)
    scene = solver.scene(sc)
    t = (12, 12, 10)

    def bad(**kw):
        a = gms.GmsArm(arm.lens, arm.base, step_cdeg=arm.step_cdeg, samples=arm.samples,
                       max_flex_cdeg=arm.max_flex_cdeg, eps=arm.eps)
        for k, v in kw.items():
            setattr(a, k, v)
        return a

    cases = [(bad(step_cdeg=7000), t), (bad(m_min=0), t), (bad(samples=0), t), (bad(samples=65), t),
             (bad(eps=-0.1), t), (bad(eps=float("nan")), t), (bad(lens=[3.0, 0.0, 3.0, 3.0]), t),
             (bad(max_flex_cdeg=(18001, 9000, 9000)), t), (bad(approach=(0, -9000, 18001)), t),
             (bad(base=(24, 0, 0)), t), (arm, (-1, 3, 3)), (arm, (3, 3, 24))]
    for a, tt in cases:
        with pytest.raises(msc.MscError) as e:
            solver.gms_reach(scene, a, tt, 4)
        assert e.value.status == msc.E_ARG
    with pytest.raises(msc.MscError) as e:
        solver.gms_reach(scene, arm, t, 0)
    assert e.value.status == msc.E_ARG


def test_gms_degenerate_settings(solver):
    """Limits at their edges, against the oracle's full solution sets: no length slack
    (eps 0), a zero-width approach cone, no flexion allowed (a straight arm), segment 1
    straight up only, and more solutions wanted than exist."""
    checked = 0
    for seed in range(3):
        arm, sc, rng = small_case(seed + 40, 2000, 24, 3)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        ts = targets_of(arm, occ, rng, 2)
        straight = (arm.base[0], arm.base[1], arm.base[2] + int(round(sum(arm.lens))))
        if straight[2] < 24 and occ[straight[2], straight[1], straight[0]] == 0:
            ts.append(np.array(straight))
        variants = [dict(eps=0.0), dict(approach=(0, -9000, 0)), dict(max_flex_cdeg=(0, 0, 0), eps=1e-6),
                    dict(seg1_min_el_cdeg=9000)]
        for kw in variants:
            a = gms.GmsArm(arm.lens, arm.base, step_cdeg=arm.step_cdeg, samples=arm.samples,
                           max_flex_cdeg=arm.max_flex_cdeg, eps=arm.eps)
            for k, v in kw.items():
                setattr(a, k, v)
            for t in ts:
                say("gms degenerate", seed, kw, tuple(t))
                compare(solver, scene, a, occ, t, want=64)
                checked += 1
    assert checked >= 24
