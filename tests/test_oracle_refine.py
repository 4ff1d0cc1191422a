"""Pins of the oracle's exact end point ("Exact IK solution with discretized segment
mappings"): the first segments keep their discrete directions, the last two are
recomputed so that the arm ends exactly on the target.  Checked by replaying the output
angles through the direction formula of the arm model, by brute-force sampling of the
circle of joints that close the triangle, and by special cases (an exact discrete end
is a fixed point, an out-of-reach target has no solution, a straight last pair)."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import synth


def fk_points(arm, ang_deg):
    """Continuous joint positions (base, after segment 1, ...) from joint angles in
    degrees: each yaw adds to the azimuth, each pitch to the elevation."""
    az, el = arm.az0_cdeg / 100.0, arm.el0_cdeg / 100.0
    p = np.array(arm.base, np.float64)
    pts = [p.copy()]
    for k, t in enumerate(arm.types):
        if t == synth.YAW:
            az += ang_deg[k]
        else:
            el += ang_deg[k]
        a, e = np.radians(az), np.radians(el)
        p = p + arm.lens[k] * np.array([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)])
        pts.append(p.copy())
    return pts


def random_case(seed, arm=None):
    rng = synth.rng_for(908, seed)
    arm = arm or synth.arm_gms()
    q = synth.candidate_poses(rng, arm, 1)[0]
    step = arm.step_cdeg / 100.0
    end = fk_points(arm, q * step)[-1]
    target = end + rng.uniform(-0.5, 0.5, size=3)
    return arm, q, target, rng


@pytest.mark.parametrize("seed", range(40))
def test_refined_arm_ends_on_target(seed):
    arm, q, target, _ = random_case(seed)
    st, ang = oracle.refine(arm, q, target)
    n = arm.dof
    step = arm.step_cdeg / 100.0
    assert np.array_equal(ang[:n - 4], q[:n - 4] * step)
    if st == oracle.OK:
        pts = fk_points(arm, ang)
        assert np.abs(pts[-1] - target).max() < 1e-9
    else:
        P = fk_points(arm, q * step)[n - 4]
        d = np.linalg.norm(target - P)
        L3, L4 = arm.lens[n - 3], arm.lens[n - 1]
        assert d > L3 + L4 or d < abs(L3 - L4)


@pytest.mark.parametrize("seed", range(40))
def test_refined_joint_is_the_closest_closing_point(seed):
    """Among all points at distance L3 from the fixed part's end P and L4 from the target
    (a circle around the line P-target), the refined joint is the one nearest the
    discrete pose's joint: checked against 7200 samples of the circle."""
    arm, q, target, _ = random_case(seed)
    st, ang = oracle.refine(arm, q, target)
    if st != oracle.OK:
        pytest.skip("no exact solution for this draw")
    n = arm.dof
    step = arm.step_cdeg / 100.0
    disc = fk_points(arm, q * step)
    got = fk_points(arm, ang)
    P, Jd, J = disc[n - 4], disc[n - 2], got[n - 2]
    L3, L4 = arm.lens[n - 3], arm.lens[n - 1]
    assert abs(np.linalg.norm(J - P) - L3) < 1e-9
    assert abs(np.linalg.norm(target - J) - L4) < 1e-9
    v = target - P
    d = np.linalg.norm(v)
    u = v / d
    c = P + u * (L3 ** 2 - L4 ** 2 + d ** 2) / (2 * d)
    rad = np.sqrt(max(L3 ** 2 - np.dot(c - P, c - P), 0.0))
    e1 = np.cross(u, [1.0, 0.0, 0.0])
    if np.linalg.norm(e1) < 0.5:
        e1 = np.cross(u, [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    th = np.linspace(0.0, 2 * np.pi, 7200, endpoint=False)
    circle = c[None, :] + rad * (np.cos(th)[:, None] * e1[None, :] + np.sin(th)[:, None] * e2[None, :])
    best = np.linalg.norm(circle - Jd[None, :], axis=1).min()
    assert np.linalg.norm(J - Jd) <= best + 1e-9
    # J lies in the plane of P, the target and Jd
    assert abs(np.dot(np.cross(target - P, Jd - P), J - P)) < 1e-6 * L3 ** 3


@pytest.mark.parametrize("seed", range(10))
def test_exact_discrete_end_is_a_fixed_point(seed):
    arm, q, _, _ = random_case(seed)
    step = arm.step_cdeg / 100.0
    end = fk_points(arm, q * step)[-1]
    st, ang = oracle.refine(arm, q, end)
    assert st == oracle.OK
    assert np.abs(ang - q * step).max() < 1e-7


def test_out_of_reach_target_has_no_exact_solution():
    arm, q, _, _ = random_case(0)
    n = arm.dof
    step = arm.step_cdeg / 100.0
    P = fk_points(arm, q * step)[n - 4]
    far = P + np.array([arm.lens[n - 3] + arm.lens[n - 1] + 0.25, 0.0, 0.0])
    st, ang = oracle.refine(arm, q, far)
    assert st == oracle.NO_REACH
    assert np.array_equal(ang, q * step)
    near = P + np.array([0.0, 0.0, abs(arm.lens[n - 3] - arm.lens[n - 1]) - 0.25])
    assert oracle.refine(arm, q, near)[0] == oracle.NO_REACH


def test_straight_last_pair_bends_to_a_closer_target():
    """The discrete last two segments in one line and the target on that line but
    nearer: the joint leaves the line (a fixed perpendicular is taken) and both lengths
    still hold."""
    arm = synth.arm_gms()
    n = arm.dof
    q = np.zeros(n, np.int64)
    q[1] = 6
    step = arm.step_cdeg / 100.0
    pts = fk_points(arm, q * step)
    P, end = pts[n - 4], pts[-1]
    target = P + (end - P) * 0.9
    st, ang = oracle.refine(arm, q, target)
    assert st == oracle.OK
    got = fk_points(arm, ang)
    assert np.abs(got[-1] - target).max() < 1e-9
    J = got[n - 2]
    assert abs(np.linalg.norm(J - P) - arm.lens[n - 3]) < 1e-9
    u = (end - P) / np.linalg.norm(end - P)
    assert np.linalg.norm((J - P) - np.dot(J - P, u) * u) > 1.0


def test_arm_shape_check():
    assert oracle.refine_ok_arm(synth.arm_gms())
    assert not oracle.refine_ok_arm(synth.arm_c2())
