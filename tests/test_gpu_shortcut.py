"""GPU parity of the short-reach shortcut and its path (msc_short_path) with the oracle,
through the C ABI: the hit (segment, sample, length, joint prefix), the status and the
rows, element by element, on tiny arms with targets on and next to their segments and
with blocked voxels before the hit point, and on 6-DOF arms on 48^3 grids; argument
errors.  Integer work: bit-exact."""
import numpy as np
import pytest

import oracle
from oracle import guided, shortcut
from paper_1906_10678_amd import msc, synth

from cases import tiny_case
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def wide(arm):
    na = 36000 // arm.step_cdeg
    arm.lo_cdeg = [-(na // 2 - 1) * arm.step_cdeg] * arm.dof
    arm.hi_cdeg = [(na // 2 - 1) * arm.step_cdeg] * arm.dof
    return arm


def compare(solver, scene, arm, occ, t, rho2, K, retries=3):
    st, rows, hit = solver.short_path(scene, arm, t, rho2, K, -1, 1, 2, 4, retries=retries)
    rst, rrows, rhit, r = shortcut.short_path(arm, occ, t, rho2, K, None, 1, 2, 4, retries=retries)
    assert st == rst, (st, rst)
    if rst == oracle.NO_REACH:
        return st, None
    assert (hit is None) == (rhit is None), (hit, rhit)
    if hit is not None:
        assert (hit["k"], hit["s"], hit["length"]) == (rhit["k"], rhit["s"], rhit["length"]), (hit, rhit)
        assert np.array_equal(hit["q"], rhit["q"]), (hit["q"], rhit["q"])
    if st == msc.OK:
        assert np.array_equal(rows, rrows)
    return st, hit


def test_short_path_tiny(solver):
    outcomes = []
    for seed in range(10):
        dof = 4 + seed % 2
        arm, sc, rng = tiny_case(seed, dof=dof)
        arm = wide(arm)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        q = synth.candidate_poses(rng, arm, 300)
        ok, ends = oracle.poses(arm, occ, q)
        for i in np.flatnonzero(ok)[:2]:
            pts = guided.sample_points(arm, q[i])
            for t in (pts[1][arm.samples // 2], pts[2][1] + np.array([0, 1, 0]), ends[i]):
                if occ[t[2], t[1], t[0]] or (t < 0).any() or (t >= occ.shape[0]).any():
                    continue
                for rho2, K in ((0, 2), (1, 3), (1, dof - 1)):
                    if not shortcut.check_radius(arm, rho2, K):
                        continue
                    say("short path tiny", seed, dof, tuple(t), rho2, K)
                    outcomes.append(compare(solver, scene, arm, occ, t, rho2, K))
    hits = [h for st, h in outcomes if h is not None]
    assert len(hits) >= 10 and any(st == msc.OK for st, h in outcomes if h is not None)


def test_short_path_blocked_before_the_hit(solver):
    seen = 0
    for seed in range(8):
        arm, sc, rng = tiny_case(seed, dof=4, nbox=0, nsph=0)
        arm = wide(arm)
        occ0 = oracle.raster(sc)
        q = synth.candidate_poses(rng, arm, 200)
        ok, _ = oracle.poses(arm, occ0, q)
        for i in np.flatnonzero(ok)[:2]:
            pts = guided.sample_points(arm, q[i])
            t, blk = pts[1][5], pts[1][2]
            if np.array_equal(t, blk) or np.array_equal(blk, pts[0][arm.samples - 1]):
                continue
            boxes = np.array([[blk[0], blk[1], blk[2], 1, 1, 1]], np.int32)
            sc2 = synth.Scene(n=sc.n, dilate=0, boxes=boxes, spheres=np.zeros((0, 4), np.int32))
            occ = oracle.raster(sc2)
            if not shortcut.check_radius(arm, 1, 3):
                continue
            say("short path blocked", seed, i)
            compare(solver, solver.scene(sc2), arm, occ, t, 1, 3)
            seen += 1
    assert seen >= 4


def test_short_path_medium(solver):
    outcomes = []
    for seed in range(4):
        rng = synth.rng_for(961, seed)
        n = 48
        arm = synth.arm_chain(6, [8, 8, 7, 6, 5, 4], 1000, 17000, (n // 2, n // 2, 0))
        sc = synth.random_scene(rng, n, 1, 6, (3, 10), 2, (2, 5), base=arm.base, column=arm.lens[0] + 2)
        occ = oracle.raster(sc)
        scene = solver.scene(sc)
        q = synth.candidate_poses(rng, arm, 400)
        ok, ends = oracle.poses(arm, occ, q)
        for i in np.flatnonzero(ok)[:2]:
            pts = guided.sample_points(arm, q[i])
            for t in (pts[2][4], ends[i]):
                say("short path medium", seed, i)
                outcomes.append(compare(solver, scene, arm, occ, t, 4, 4)[0])
    assert msc.OK in outcomes


def test_short_path_argument_errors(solver):
    arm, sc, rng = tiny_case(2, dof=4)
    arm = wide(arm)
    scene = solver.scene(sc)
    t = (sc.n // 2, sc.n // 2, 3)
    for rho2, K in ((1, 1), (1, 4), (-1, 2), (10 ** 6, 2)):
        with pytest.raises(msc.MscError) as e:
            solver.short_path(scene, arm, t, rho2, K)
        assert e.value.status == msc.E_ARG
