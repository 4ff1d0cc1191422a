"""Pins of the oracle's segment tables against closed-form values and exact symmetries.

A segment of length L with global azimuth az and elevation el maps by
L * (cos el cos az, cos el sin az, sin el) (eq 1 and its vector-sum form, with the
quiver directions in the global frame, section "Discretization of the segment
articulations"); the mapping is rounded back onto the voxel grid (section "The
representations of the arm and obstacles"), exact halves away from zero.
"""
import math

import numpy as np
import pytest

import oracle


def off_of(L, az_deg, el_deg, step_deg=5):
    na = int(round(360 / step_deg))
    off, _ = oracle.tables(na, 8, L)
    ia = int(round(az_deg / step_deg)) % na
    ie = int(round(el_deg / step_deg)) % na
    return tuple(int(v) for v in off[ia, ie])


# Hand-computed with exact trigonometric values (cos 60 = 1/2, cos 45 = sqrt2/2 ...).
HAND = [
    # L, az, el, expected offset, arithmetic
    (10, 0, 0, (10, 0, 0), "10*(1,0,0)"),
    (10, 0, 90, (0, 0, 10), "cos 90 = 0"),
    (10, 135, 90, (0, 0, 10), "vertical for every azimuth"),
    (10, 45, 0, (7, 7, 0), "10*0.7071 = 7.07"),
    (25, 60, 0, (13, 22, 0), "25/2 = 12.5 is a tie -> 13; 25*0.8660 = 21.65 -> 22"),
    (25, 0, 30, (22, 0, 13), "21.65 -> 22; 25*sin30 = 12.5 tie -> 13"),
    (10, 60, 60, (3, 4, 9), "10/4 = 2.5 tie -> 3; 10*0.5*0.866 = 4.33; 8.66 -> 9"),
    (8, 0, -30, (7, 0, -4), "8*0.866 = 6.93 -> 7; -4 exactly"),
    (6, 180, 45, (-4, 0, 4), "6*0.7071 = 4.24 -> -4 and 4"),
    (5, 45, 45, (3, 3, 4), "5/2 = 2.5 ties -> 3, 3; 3.54 -> 4"),
    (12, 90, 0, (0, 12, 0), "(cos 90, sin 90) = (0, 1)"),
    (12, 270, 0, (0, -12, 0), ""),
    (30, 0, 180, (-30, 0, 0), "cos 180 = -1, sin 180 = 0"),
    (20, 30, 60, (9, 5, 17), "20*0.5*0.866 = 8.66 -> 9; 20*0.5*0.5 = 5; 17.32 -> 17"),
]


@pytest.mark.parametrize("L,az,el,expect,why", HAND)
def test_hand_values(L, az, el, expect, why):
    assert off_of(L, az, el) == expect, why


def test_sweep_hand_value():
    # L = 30, az = 0, el = 60, sample 1 of 8 lies at 30/8 = 3.75 along the segment:
    # (3.75*0.5, 0, 3.75*0.8660) = (1.875, 0, 3.248) -> (2, 0, 3).
    off, sweep = oracle.tables(72, 8, 30)
    assert tuple(sweep[0, 12, 0]) == (2, 0, 3)
    # sample S is the segment end
    assert np.array_equal(sweep[:, :, 7, :], off)


def test_zero_length_segment():
    off, sweep = oracle.tables(36, 8, 0)
    assert not off.any() and not sweep.any()


@pytest.mark.parametrize("na", [8, 12, 36, 72, 144])
@pytest.mark.parametrize("L", [1, 5, 10, 25, 30, 60])
def test_exact_symmetries(na, L):
    """Mirror / rotation symmetries of the direction map hold entry by entry because
    the rounding is odd (halves away from zero)."""
    off, sweep = oracle.tables(na, 8, L)
    idx = np.arange(na)
    neg = (-idx) % na
    half = (idx + na // 2) % na
    quarter_minus = (na // 4 - idx) % na
    for T in (off, sweep[:, :, 2, :], sweep[:, :, 5, :]):
        x, y, z = T[..., 0], T[..., 1], T[..., 2]
        # off(-az, el) = (x, -y, z)
        m = T[neg, :, :]
        assert np.array_equal(m[..., 0], x) and np.array_equal(m[..., 1], -y) and np.array_equal(m[..., 2], z)
        # off(az + 180, el) = (-x, -y, z)
        m = T[half, :, :]
        assert np.array_equal(m[..., 0], -x) and np.array_equal(m[..., 1], -y) and np.array_equal(m[..., 2], z)
        # off(az, -el) = (x, y, -z)
        m = T[:, neg, :]
        assert np.array_equal(m[..., 0], x) and np.array_equal(m[..., 1], y) and np.array_equal(m[..., 2], -z)
        if na % 4 == 0:
            # off(90 - az, el) = (y, x, z)
            m = T[quarter_minus, :, :]
            assert np.array_equal(m[..., 0], y) and np.array_equal(m[..., 1], x) and np.array_equal(m[..., 2], z)


@pytest.mark.parametrize("na,L", [(36, 10), (72, 30), (72, 25), (144, 60)])
def test_within_half_voxel_diagonal(na, L):
    """Each rounded coordinate is within 1/2 of the real one, so every entry lies within
    sqrt(3)/2 of L*d(o); computed here with numpy's own trigonometry in degrees."""
    off, sweep = oracle.tables(na, 8, L)
    deg = np.arange(na) * 360.0 / na
    az = np.radians(deg)[:, None]
    el = np.radians(deg)[None, :]
    real = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el) * np.ones_like(az)], -1)
    assert np.all(np.abs(off - L * real) <= 0.5 + 1e-9)
    for s in range(1, 9):
        assert np.all(np.abs(sweep[:, :, s - 1, :] - (s * L / 8.0) * real) <= 0.5 + 1e-9)


@pytest.mark.parametrize("na,lens", [(36, [10, 8, 6]), (72, [30, 25, 20, 15, 10]), (144, [60, 50, 40, 30, 20])])
def test_tie_band_is_never_borderline(na, lens):
    """The rounding treats |frac - 1/2| <= 1e-9 as an exact tie.  For every table entry
    of the workload arms the distance to a half-integer is either below 1e-11 (a true
    tie, rational cos/sin products) or above 1e-6, so no FP64 evaluation order can move
    an entry across the band."""
    deg = np.arange(na) * 360.0 / na
    az = np.radians(deg)[:, None]
    el = np.radians(deg)[None, :]
    dirs = [np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el) * np.ones_like(az)]
    for L in lens:
        for s in range(1, 9):
            c = s * L / 8.0
            for d in dirs:
                v = np.abs(c * d)
                dist = np.abs(v - np.floor(v) - 0.5)
                assert np.all((dist < 1e-11) | (dist > 1e-6))


def test_reach_radii():
    """ceil(max |off|): the vertical direction is in every table (norm exactly L) and a
    rounded offset is within sqrt(3)/2 of its real vector, so L <= radius <= L + 1;
    (13, 22, 0) for L = 25 at 60 deg has norm 25.55, so that radius is 26."""
    from paper_1906_10678_amd import synth
    arm = synth.arm_c2()
    radii = list(oracle.reach_radii(arm))
    for L, R in zip(arm.lens, radii):
        assert L <= R <= L + 1
    assert radii[2] == 26
