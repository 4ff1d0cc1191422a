"""Oracle of the paper's gap map-seeking search: the quiver tiling of the sphere and the
four-segment search with a free vector across the gap.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the GPU library or its
binding.  It shares no code with the GPU path.  Plain Python / numpy in FP64; the
trigonometry of the quiver uses ``math`` (the platform's libm), angles converted as
(degrees * pi) / 180.

Readings of "Discretization of the segment articulations", "The gap in gMS" (eqs 2-8),
"Exact IK solution with discretized segment mappings", "Testing for collisions" and
"The procedure for IK solution":

* Quiver of step D degrees (D divides 180; n = 360 / D azimuths on the equator):
  elevations e_i = -90 + i D, i = 0..180/D, equidistant; at e_i the ring has
  m_i = 1 vector at the poles, else max(m_min, round(n cos e_i)) (the equatorial
  great-circle spacing kept along the ring; halves away from zero, a value within 1e-9
  of a half counts as one), azimuths a_ij = (j * 360) / m_i.  Vector (cos e cos a,
  cos e sin a, sin e); flat index = vectors of the rings below + j ([elevation order,
  azimuth order]).
* Arm: four segments of lengths L1..L4 (voxels, reals), each pointing along a quiver
  vector of the global frame except segment 3, the free vector v3 that spans the gap
  from the end p2 of segment 2 to the start p3 = t - L4 r_l of segment 4.  Constraints:
  segment 1's elevation at least e_min1 (upper hemisphere, say); the flexion between
  consecutive segments at most theta_1, theta_2, theta_3 (u_k . u_{k+1} >= cos theta - 1e-9,
  for the free vector decided on squares without a square root: see flex_ok); segment 4
  inside the approach cone (r_l . a >= cos alpha - 1e-9) or, with alpha < 0, every
  quiver vector; |v3| within eps of L3, decided as (L3 - eps)^2 <= |v3|^2 <= (L3 + eps)^2.
* Positions stay numerical: p1 = p0 + L1 r_i, p2 = p1 + L2 r_j, component by component,
  one multiply and one add each.  A segment from p along w is clear when its samples
  p + (s / S) w, s = 1..S, rounded per component (halves away from zero, 1e-9 band), are
  inside the grid and free.
* Pruning (eqs 5-8, widened by eps so that no solution is lost): |p1 - t|^2 <=
  (L2 + L3 + L4 + eps)^2; |p2 - t|^2 <= (L3 + L4 + eps)^2 (bounds squared as b * b).
* Steps 1, 2A, 2B: survivors of segment 1; then segment 2 from each; then every segment-4
  vector that is clear on its own; a triple (i, j, l) is a solution when all tests pass.
  The reach pose is the first solution in (i, j, l) order.  The exact end point of the
  8-DOF text: s3 = v3 L3 / |v3|, s4' = (t - p2) - s3.

Parity status: pinned in tests/test_oracle_gms_quiver.py: the quiver against its closed
form (ring counts, unit length, exact vectors at the poles and the equator, mirror
symmetry), the pruned search against the unpruned enumeration of every (i, j, l), each
solution against a plain replay of its constraints, and the exact end point.
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np

BAND = 1e-9


def round_half_away(v: float) -> int:
    a = abs(v)
    f = math.floor(a)
    frac = a - f
    r = f + 1 if (frac > 0.5 or abs(frac - 0.5) <= BAND) else f
    return int(r) if v >= 0 else -int(r)


def _rad(deg: float) -> float:
    return (deg * math.pi) / 180.0


def quiver(step_cdeg: int, m_min: int = 4) -> np.ndarray:
    """Quiver unit vectors (count, 3) in flat index order."""
    if 18000 % step_cdeg:
        raise ValueError("the step must divide 180 degrees")
    D = step_cdeg / 100.0
    n = 36000 // step_cdeg
    out = []
    for i in range(18000 // step_cdeg + 1):
        e = -90.0 + i * D
        if abs(e) == 90.0:
            m = 1
        else:
            m = max(m_min, round_half_away(n * math.cos(_rad(e))))
        ce, se = math.cos(_rad(e)), math.sin(_rad(e))
        for j in range(m):
            a = (j * 360.0) / m
            out.append((ce * math.cos(_rad(a)), ce * math.sin(_rad(a)), se))
    return np.array(out, np.float64)


def ring_counts(step_cdeg: int, m_min: int = 4) -> List[int]:
    D = step_cdeg / 100.0
    n = 36000 // step_cdeg
    counts = []
    for i in range(18000 // step_cdeg + 1):
        e = -90.0 + i * D
        counts.append(1 if abs(e) == 90.0 else max(m_min, round_half_away(n * math.cos(_rad(e)))))
    return counts


class GmsArm:
    """Four-segment arm of the gap search (all angles in centidegrees)."""

    def __init__(self, lens, base, step_cdeg=200, m_min=4, samples=8, seg1_min_el_cdeg=0,
                 max_flex_cdeg=(13500, 13500, 13500), approach=None, eps=0.5):
        self.lens = [float(v) for v in lens]
        self.base = tuple(int(v) for v in base)
        self.step_cdeg = step_cdeg
        self.m_min = m_min
        self.samples = samples
        self.seg1_min_el_cdeg = seg1_min_el_cdeg
        self.max_flex_cdeg = tuple(max_flex_cdeg)
        self.approach = approach          # (az_cdeg, el_cdeg, half_cdeg) or None
        self.eps = float(eps)


def _unit(az_cdeg, el_cdeg):
    a, e = _rad(az_cdeg / 100.0), _rad(el_cdeg / 100.0)
    return np.array([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)])


def _clear(occ, p, w, S) -> bool:
    N = occ.shape[0]
    for s in range(1, S + 1):
        t = s / S
        v = [round_half_away(p[c] + t * w[c]) for c in range(3)]
        if min(v) < 0 or max(v) >= N or occ[v[2], v[1], v[0]]:
            return False
    return True


def _cosl(cdeg):
    return math.cos(_rad(cdeg / 100.0)) - BAND


def _norm(v) -> float:
    return math.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])


def _dot(a, b) -> float:
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _add(p, L, r):
    return (p[0] + L * r[0], p[1] + L * r[1], p[2] + L * r[2])


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def gap_bounds(L3: float, eps: float):
    """Squared bounds of the free vector's length: |v3| within eps of L3."""
    lo = max(L3 - eps, 0.0)
    hi = L3 + eps
    return lo * lo, hi * hi


def flex_ok(dot: float, c: float, n2: float) -> bool:
    """u . v >= c |v| for a unit u, decided on squares: dot >= 0 and dot^2 >= c^2 |v|^2
    when c >= 0; dot >= 0 or dot^2 <= c^2 |v|^2 when c < 0."""
    if c >= 0:
        return dot >= 0 and dot * dot >= (c * c) * n2
    return dot >= 0 or dot * dot <= (c * c) * n2


def _flex_arr(dot: np.ndarray, c: float, n2: np.ndarray) -> np.ndarray:
    if c >= 0:
        return (dot >= 0) & (dot * dot >= (c * c) * n2)
    return (dot >= 0) | (dot * dot <= (c * c) * n2)


def seg4_set(arm: GmsArm, occ, target, Q) -> List[int]:
    """Segment-4 vectors l inside the cone whose segment is clear on its own."""
    L4 = arm.lens[3]
    t = tuple(float(v) for v in target)
    axis = None if arm.approach is None else _unit(arm.approach[0], arm.approach[1])
    out = []
    for l in range(len(Q)):
        r = tuple(Q[l])
        if axis is not None and _dot(r, axis) < _cosl(arm.approach[2]):
            continue
        p3 = (t[0] - L4 * r[0], t[1] - L4 * r[1], t[2] - L4 * r[2])
        if _clear(occ, p3, (L4 * r[0], L4 * r[1], L4 * r[2]), arm.samples):
            out.append(l)
    return out


def solutions_plain(arm: GmsArm, occ, target, prune: bool = True,
                    limit: Optional[int] = None) -> List[Tuple[int, int, int]]:
    """Every solution (i, j, l) in order (Steps 1, 2A, 2B), one hypothesis at a time;
    prune=False skips eqs 5-8 (the result must not change).  Tiny quivers only."""
    Q = quiver(arm.step_cdeg, arm.m_min)
    Qt = [tuple(v) for v in Q]
    L1, L2, L3, L4 = arm.lens
    eps, S = arm.eps, arm.samples
    p0 = tuple(float(v) for v in arm.base)
    t = tuple(float(v) for v in target)
    N = occ.shape[0]
    tv = [int(v) for v in target]
    if min(tv) < 0 or max(tv) >= N or occ[tv[2], tv[1], tv[0]]:
        return []
    b = [int(v) for v in arm.base]
    if occ[b[2], b[1], b[0]]:
        return []
    ls = seg4_set(arm, occ, target, Q)
    min_el = math.sin(_rad(arm.seg1_min_el_cdeg / 100.0)) - BAND
    c1, c2, c3 = (_cosl(v) for v in arm.max_flex_cdeg)
    g_lo, g_hi = gap_bounds(L3, eps)
    r5, r7 = L2 + L3 + L4 + eps, L3 + L4 + eps
    out = []
    for i, ri in enumerate(Qt):
        if ri[2] < min_el:                                   # joint 1 limit
            continue
        p1 = _add(p0, L1, ri)
        if prune:
            d = _sub(p1, t)
            if _dot(d, d) > r5 * r5:                          # eq 5
                continue
        if not _clear(occ, p0, (L1 * ri[0], L1 * ri[1], L1 * ri[2]), S):
            continue
        for j, rj in enumerate(Qt):
            if _dot(ri, rj) < c1:                            # joint 2 limit
                continue
            p2 = _add(p1, L2, rj)
            if prune:
                d = _sub(p2, t)
                if _dot(d, d) > r7 * r7:                      # eq 7
                    continue
            if not _clear(occ, p1, (L2 * rj[0], L2 * rj[1], L2 * rj[2]), S):
                continue
            for l in ls:
                rl = Qt[l]
                p3 = (t[0] - L4 * rl[0], t[1] - L4 * rl[1], t[2] - L4 * rl[2])
                v3 = _sub(p3, p2)
                n2 = _dot(v3, v3)
                if n2 < g_lo or n2 > g_hi:                   # the gap's free vector
                    continue
                if not flex_ok(_dot(rj, v3), c2, n2):        # joint 3 limit
                    continue
                if not flex_ok(_dot(v3, rl), c3, n2):        # joint 4 limit
                    continue
                if not _clear(occ, p2, v3, S):
                    continue
                out.append((i, j, l))
                if limit is not None and len(out) >= limit:
                    return out
    return out


def _round_arr(v: np.ndarray) -> np.ndarray:
    a = np.abs(v)
    f = np.floor(a)
    frac = a - f
    r = np.where((frac > 0.5) | (np.abs(frac - 0.5) <= BAND), f + 1, f)
    return np.where(v >= 0, r, -r).astype(np.int64)


def _clear_arr(occ, p: np.ndarray, w: np.ndarray, S: int) -> np.ndarray:
    """Segments from p[m, 3] along w[m, 3]: clear flags [m] (same arithmetic as _clear)."""
    N = occ.shape[0]
    ok = np.ones(len(p), bool)
    for s in range(1, S + 1):
        t = s / S
        v = _round_arr(p + t * w)
        inside = ((v >= 0) & (v < N)).all(axis=1)
        c = np.clip(v, 0, N - 1)
        ok &= inside & (occ[c[:, 2], c[:, 1], c[:, 0]] == 0)
    return ok


def solutions(arm: GmsArm, occ, target, limit: Optional[int] = None) -> List[Tuple[int, int, int]]:
    """The same solutions as solutions_plain (with pruning), the hypotheses of one
    segment-1 vector at a time held in numpy arrays (each element computed with the same
    operations in the same order)."""
    Q = quiver(arm.step_cdeg, arm.m_min)
    L1, L2, L3, L4 = arm.lens
    eps, S = arm.eps, arm.samples
    p0 = np.array(arm.base, np.float64)
    t = np.array(target, np.float64)
    N = occ.shape[0]
    tv = [int(v) for v in target]
    if min(tv) < 0 or max(tv) >= N or occ[tv[2], tv[1], tv[0]]:
        return []
    b = [int(v) for v in arm.base]
    if occ[b[2], b[1], b[0]]:
        return []
    ls = np.array(seg4_set(arm, occ, target, Q), np.int64)
    if len(ls) == 0:
        return []
    RL = Q[ls]
    P3 = t[None, :] - L4 * RL
    min_el = math.sin(_rad(arm.seg1_min_el_cdeg / 100.0)) - BAND
    c1, c2, c3 = (_cosl(v) for v in arm.max_flex_cdeg)
    g_lo, g_hi = gap_bounds(L3, eps)
    r5, r7 = L2 + L3 + L4 + eps, L3 + L4 + eps
    out = []
    for i in range(len(Q)):
        ri = Q[i]
        if ri[2] < min_el:
            continue
        p1 = p0 + L1 * ri
        d = p1 - t
        if _dot(d, d) > r5 * r5:
            continue
        if not _clear_arr(occ, p0[None, :], (L1 * ri)[None, :], S)[0]:
            continue
        dots = Q[:, 0] * ri[0] + Q[:, 1] * ri[1] + Q[:, 2] * ri[2]
        js = np.flatnonzero(dots >= c1)
        P2 = p1[None, :] + L2 * Q[js]
        d = P2 - t[None, :]
        dd = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        keep = dd <= r7 * r7
        js, P2 = js[keep], P2[keep]
        if len(js) == 0:
            continue
        keep = _clear_arr(occ, np.repeat(p1[None, :], len(js), axis=0), L2 * Q[js], S)
        js, P2 = js[keep], P2[keep]
        for jj in range(len(js)):
            j, p2 = int(js[jj]), P2[jj]
            rj = Q[j]
            V3 = P3 - p2[None, :]
            n2 = V3[:, 0] * V3[:, 0] + V3[:, 1] * V3[:, 1] + V3[:, 2] * V3[:, 2]
            ok = (n2 >= g_lo) & (n2 <= g_hi)
            ok &= _flex_arr(rj[0] * V3[:, 0] + rj[1] * V3[:, 1] + rj[2] * V3[:, 2], c2, n2)
            ok &= _flex_arr(V3[:, 0] * RL[:, 0] + V3[:, 1] * RL[:, 1] + V3[:, 2] * RL[:, 2], c3, n2)
            cand = np.flatnonzero(ok)
            if len(cand) == 0:
                continue
            cl = _clear_arr(occ, np.repeat(p2[None, :], len(cand), axis=0), V3[cand], S)
            for l in ls[cand[cl]]:
                out.append((i, j, int(l)))
                if limit is not None and len(out) >= limit:
                    return out
    return out


def vectors(arm: GmsArm, target, sol) -> np.ndarray:
    """(6, 3): s1, s2, v3, s4 of solution (i, j, l), then the exact s3, s4' of the 8-DOF
    text (s3 = v3 L3 / |v3|, s4' = (t - p2) - s3)."""
    Q = quiver(arm.step_cdeg, arm.m_min)
    L1, L2, L3, L4 = arm.lens
    i, j, l = sol
    ri, rj, rl = tuple(Q[i]), tuple(Q[j]), tuple(Q[l])
    p0 = tuple(float(v) for v in arm.base)
    t = tuple(float(v) for v in target)
    p1 = _add(p0, L1, ri)
    p2 = _add(p1, L2, rj)
    p3 = (t[0] - L4 * rl[0], t[1] - L4 * rl[1], t[2] - L4 * rl[2])
    v3 = _sub(p3, p2)
    n3 = _norm(v3)
    s3 = tuple(v3[c] * L3 / n3 for c in range(3))
    d3 = _sub(t, p2)
    s4e = _sub(d3, s3)
    return np.array([(L1 * ri[0], L1 * ri[1], L1 * ri[2]), (L2 * rj[0], L2 * rj[1], L2 * rj[2]), v3,
                     (L4 * rl[0], L4 * rl[1], L4 * rl[2]), s3, s4e], np.float64)
