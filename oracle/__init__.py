"""CPU oracle for the staged reach search and the tube path search.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.  It
shares no code with the GPU path.  The staged sets, tables, raster and pose replay
are plain C++ (``msc_oracle.cpp``, built into ``liborc.so`` with ``g++ -O2``);
the tube path search of ``plan_path`` is plain numpy with scipy's binary maximum
filter as the one library step.

Arm objects are duck-typed: anything with ``types, lens, lo_cdeg, hi_cdeg,
step_cdeg, base, samples, az0_cdeg, el0_cdeg``.  Scenes: ``n, dilate, boxes,
spheres``.  Joint values are integer steps.

Parity status: every function here is pinned by tests in ``tests/test_oracle_*``
(closed forms, brute force, invariants).  The paper prints no worked numeric
example, so no value is pinned to the paper itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np
from scipy import ndimage

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msc_oracle.cpp")
_LIB = os.path.join(_HERE, "liborc.so")

OK, NO_REACH, NO_PATH = 0, 1, 2
E_ARG = -1


def build(force: bool = False) -> str:
    """Compile the oracle with g++ -O2 (plain scalar code, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Arm(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("na", ctypes.c_int32), ("S", ctypes.c_int32),
                ("base", ctypes.c_int32 * 3), ("ia0", ctypes.c_int32), ("ie0", ctypes.c_int32),
                ("type", ctypes.c_int32 * 16), ("len", ctypes.c_int32 * 16),
                ("lo", ctypes.c_int32 * 16), ("hi", ctypes.c_int32 * 16),
                ("ref", ctypes.c_int32 * 16),
                ("app_az_cdeg", ctypes.c_int32), ("app_el_cdeg", ctypes.c_int32), ("app_half_cdeg", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        L.orc_tables.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
        L.orc_raster.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32,
                                 P(ctypes.c_int32), ctypes.c_int32, P(ctypes.c_uint8)]
        L.orc_pose.argtypes = [P(_Arm), ctypes.c_int32, P(ctypes.c_uint8), P(ctypes.c_int32),
                               P(ctypes.c_int64), P(ctypes.c_int64)]
        L.orc_pose_batch.argtypes = [P(_Arm), ctypes.c_int32, P(ctypes.c_uint8), P(ctypes.c_int32),
                                     ctypes.c_int64, P(ctypes.c_uint8), P(ctypes.c_int64)]
        L.orc_pose_continuous.argtypes = [P(_Arm), P(ctypes.c_int32), P(ctypes.c_double)]
        L.orc_orientations.argtypes = [P(_Arm), P(ctypes.c_uint8)]
        L.orc_reach_radii.argtypes = [P(_Arm), P(ctypes.c_int64)]
        L.orc_solve.argtypes = [P(_Arm), ctypes.c_int32, P(ctypes.c_uint8), P(ctypes.c_int32),
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.orc_solve.restype = ctypes.c_void_p
        for f in ("orc_status", "orc_split", "orc_nsol"):
            getattr(L, f).argtypes = [ctypes.c_void_p]
        L.orc_sols.argtypes = [ctypes.c_void_p, P(ctypes.c_int32)]
        L.orc_set.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_uint64)]
        L.orc_set.restype = ctypes.c_int64
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_brute_sets.argtypes = [P(_Arm), ctypes.c_int32, P(ctypes.c_uint8), P(ctypes.c_int32),
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.orc_brute_set.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_uint64)]
        L.orc_brute_set.restype = ctypes.c_int64
        L.orc_brute_solutions.argtypes = [P(_Arm), ctypes.c_int32, P(ctypes.c_uint8), P(ctypes.c_int32),
                                          ctypes.c_int64, P(ctypes.c_int32)]
        L.orc_brute_solutions.restype = ctypes.c_int64
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def make_arm(arm, lo: Optional[Sequence[int]] = None, hi: Optional[Sequence[int]] = None,
             ref: Optional[Sequence[int]] = None, approach=None) -> _Arm:
    """Oracle arm from a duck-typed arm; lo/hi/ref override the limits (steps);
    approach = (az_cdeg, el_cdeg, half_cdeg) restricts the last segment's direction."""
    n = len(arm.types)
    step = arm.step_cdeg
    a = _Arm()
    a.n = n
    a.na = 36000 // step
    a.S = arm.samples
    for c in range(3):
        a.base[c] = int(arm.base[c])
    a.ia0 = arm.az0_cdeg // step
    a.ie0 = arm.el0_cdeg // step
    for k in range(n):
        a.type[k] = int(arm.types[k])
        a.len[k] = int(arm.lens[k])
        a.lo[k] = int(lo[k]) if lo is not None else int(arm.lo_cdeg[k] // step)
        a.hi[k] = int(hi[k]) if hi is not None else int(arm.hi_cdeg[k] // step)
        a.ref[k] = int(ref[k]) if ref is not None else 0
    a.app_az_cdeg, a.app_el_cdeg, a.app_half_cdeg = (0, 0, -1) if approach is None else (int(v) for v in approach)
    return a


# --------------------------------------------------------------------------
# Tables, raster, pose replay
# --------------------------------------------------------------------------

def tables(na: int, samples: int, length: int) -> Tuple[np.ndarray, np.ndarray]:
    """off[ia, ie, 3] and sweep[ia, ie, s-1, 3] (int32) of one segment."""
    off = np.zeros((na, na, 3), np.int32)
    sweep = np.zeros((na, na, samples, 3), np.int32)
    rc = lib().orc_tables(na, samples, length, _ptr(off, ctypes.c_int32), _ptr(sweep, ctypes.c_int32))
    assert rc == 0
    return off, sweep


def raster(scene) -> np.ndarray:
    """Blocked-voxel grid occ[z, y, x] (uint8, 1 = blocked)."""
    n = scene.n
    occ = np.zeros((n, n, n), np.uint8)
    boxes = np.ascontiguousarray(np.asarray(scene.boxes, np.int32).reshape(-1, 6))
    sph = np.ascontiguousarray(np.asarray(scene.spheres, np.int32).reshape(-1, 4))
    rc = lib().orc_raster(n, scene.dilate, _ptr(boxes, ctypes.c_int32), boxes.shape[0],
                          _ptr(sph, ctypes.c_int32), sph.shape[0], _ptr(occ, ctypes.c_uint8))
    assert rc == 0
    return occ


def poses(arm, occ: np.ndarray, q: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Replay poses q[count, dof]: (valid[count] bool, end[count, 3] int64)."""
    q = np.ascontiguousarray(np.asarray(q, np.int32).reshape(-1, len(arm.types)))
    occ = np.ascontiguousarray(occ, np.uint8)
    a = make_arm(arm)
    valid = np.zeros(q.shape[0], np.uint8)
    ends = np.zeros((q.shape[0], 3), np.int64)
    lib().orc_pose_batch(ctypes.byref(a), occ.shape[0], _ptr(occ, ctypes.c_uint8), _ptr(q, ctypes.c_int32),
                         q.shape[0], _ptr(valid, ctypes.c_uint8), _ptr(ends, ctypes.c_int64))
    return valid.astype(bool), ends


def pose_joints(arm, occ: np.ndarray, q: Sequence[int]) -> Tuple[bool, np.ndarray]:
    """Replay one pose: (valid, joint voxels[(dof+1), 3], base first)."""
    qq = np.ascontiguousarray(np.asarray(q, np.int32))
    a = make_arm(arm)
    joints = np.zeros((len(arm.types) + 1, 3), np.int64)
    end = np.zeros(3, np.int64)
    ok = lib().orc_pose(ctypes.byref(a), occ.shape[0], _ptr(np.ascontiguousarray(occ), ctypes.c_uint8),
                        _ptr(qq, ctypes.c_int32), _ptr(end, ctypes.c_int64), _ptr(joints, ctypes.c_int64))
    return bool(ok), joints


def pose_continuous(arm, q: Sequence[int]) -> np.ndarray:
    qq = np.ascontiguousarray(np.asarray(q, np.int32))
    a = make_arm(arm)
    end = np.zeros(3, np.float64)
    lib().orc_pose_continuous(ctypes.byref(a), _ptr(qq, ctypes.c_int32), _ptr(end, ctypes.c_double))
    return end


def orientations(arm, lo=None, hi=None) -> np.ndarray:
    """O_k for k = 0..n as bool[n+1, na, na]."""
    a = make_arm(arm, lo, hi)
    out = np.zeros((a.n + 1, a.na, a.na), np.uint8)
    lib().orc_orientations(ctypes.byref(a), _ptr(out, ctypes.c_uint8))
    return out.astype(bool)


def reach_radii(arm) -> np.ndarray:
    a = make_arm(arm)
    out = np.zeros(a.n, np.int64)
    lib().orc_reach_radii(ctypes.byref(a), _ptr(out, ctypes.c_int64))
    return out


def pose_fn_for(arm, scene):
    """A synth-compatible pose function backed by the oracle."""
    occ = raster(scene)

    def f(q):
        return poses(arm, occ, q)

    return f


# --------------------------------------------------------------------------
# Staged reach search
# --------------------------------------------------------------------------

class ReachResult:
    def __init__(self, status: int, m: int, sols: np.ndarray, sets: dict):
        self.status = status
        self.m = m
        self.sols = sols          # [nsol, dof] canonical order
        self.sets = sets          # {("F", k): keys, ("B", k): keys, ("C", m): keys, ("D", k): keys}

    @property
    def pose(self) -> Optional[np.ndarray]:
        return self.sols[0] if len(self.sols) else None


def reach(arm, occ: np.ndarray, target: Sequence[int], m: Optional[int] = None, want: int = 1,
          lo=None, hi=None, ref=None, prune: bool = True, keep_sets: bool = True, approach=None) -> ReachResult:
    """Staged forward/backward search with exact per-stage de-duplication; returns
    the first ``want`` solutions in the canonical order and (optionally) every set.
    Keys: (voxel (z*N+y)*N+x) << 16 | ia << 8 | ie."""
    a = make_arm(arm, lo, hi, ref, approach)
    n = a.n
    if m is None:
        m = (n + 1) // 2
    occ = np.ascontiguousarray(occ, np.uint8)
    t = np.ascontiguousarray(np.asarray(target, np.int32))
    L = lib()
    h = L.orc_solve(ctypes.byref(a), occ.shape[0], _ptr(occ, ctypes.c_uint8), _ptr(t, ctypes.c_int32),
                    m, want, 1 if prune else 0)
    if not h:
        raise ValueError("bad arguments")
    try:
        status = L.orc_status(h)
        nsol = L.orc_nsol(h)
        sols = np.zeros((nsol, n), np.int32)
        if nsol:
            L.orc_sols(h, _ptr(sols, ctypes.c_int32))
        sets = {}
        if keep_sets:
            def get(which, stage):
                cnt = L.orc_set(h, which, stage, None)
                if cnt < 0:
                    return None
                out = np.zeros(cnt, np.uint64)
                if cnt:
                    L.orc_set(h, which, stage, _ptr(out, ctypes.c_uint64))
                return out
            for k in range(m + 1):
                sets[("F", k)] = get(0, k)
                sets[("D", k)] = get(3, k)
            for k in range(m, n + 1):
                sets[("B", k)] = get(1, k)
            sets[("C", m)] = get(2, 0)
        return ReachResult(status, m, sols, sets)
    finally:
        L.orc_free(h)


def brute_sets(arm, occ, target, kf: int, kb: int, prune: bool = True, lo=None, hi=None, approach=None):
    """Per-stage sets by exhaustive enumeration of prefixes (forward, stages 0..kf)
    and suffixes (backward, stages kb..n).  Tiny arms only."""
    a = make_arm(arm, lo, hi, approach=approach)
    occ = np.ascontiguousarray(occ, np.uint8)
    t = np.ascontiguousarray(np.asarray(target, np.int32))
    L = lib()
    rc = L.orc_brute_sets(ctypes.byref(a), occ.shape[0], _ptr(occ, ctypes.c_uint8), _ptr(t, ctypes.c_int32),
                          kf, kb, 1 if prune else 0)
    out = {}
    if rc != 0:
        return out
    for k in range(kf + 1):
        cnt = L.orc_brute_set(0, k, None)
        v = np.zeros(cnt, np.uint64)
        if cnt:
            L.orc_brute_set(0, k, _ptr(v, ctypes.c_uint64))
        out[("F", k)] = v
    for k in range(kb, a.n + 1):
        cnt = L.orc_brute_set(1, k, None)
        v = np.zeros(cnt, np.uint64)
        if cnt:
            L.orc_brute_set(1, k, _ptr(v, ctypes.c_uint64))
        out[("B", k)] = v
    return out


def brute_solutions(arm, occ, target, cap: int = 1 << 20, lo=None, hi=None, ref=None):
    """(count, first min(cap, count) solutions in canonical order) by exhaustive
    replay of every joint tuple.  Tiny arms only."""
    a = make_arm(arm, lo, hi, ref)
    occ = np.ascontiguousarray(occ, np.uint8)
    t = np.ascontiguousarray(np.asarray(target, np.int32))
    out = np.zeros((cap, a.n), np.int32)
    cnt = lib().orc_brute_solutions(ctypes.byref(a), occ.shape[0], _ptr(occ, ctypes.c_uint8),
                                    _ptr(t, ctypes.c_int32), cap, _ptr(out, ctypes.c_int32))
    return int(cnt), out[:min(cap, cnt)]


# --------------------------------------------------------------------------
# Path: reach pose first, then a tube search over the waypoints
# --------------------------------------------------------------------------

def guide(start: np.ndarray, goal: np.ndarray, W: int) -> np.ndarray:
    """g[w] = start + round_half_away(w * (goal - start) / W) in integers, w = 0..W."""
    D = np.asarray(goal, np.int64) - np.asarray(start, np.int64)
    g = np.zeros((W + 1, len(D)), np.int64)
    for w in range(W + 1):
        num = w * D
        mag = (2 * np.abs(num) + W) // (2 * W)
        g[w] = np.asarray(start, np.int64) + np.sign(num) * mag
    return g


def _box_poses(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    axes = [np.arange(lo[k], hi[k] + 1) for k in range(len(lo))]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1).astype(np.int32)


def tube_search(arm, occ, start, goal, W: int, delta: int, r: int, lim_lo, lim_hi):
    """Waypoint tube search ("Smooth sequence computation"; "Filtering for
    smoothness"): poses within r steps of the guide at every waypoint, each move
    changing every joint by at most delta; the sequence is chosen backward from the
    reach pose, at each waypoint the pose closest (L1) to the guide, ties by joint
    values.  Returns the (W+1, dof) path or None."""
    dof = len(start)
    start = np.asarray(start, np.int64)
    goal = np.asarray(goal, np.int64)
    g = guide(start, goal, W)
    lo_b, hi_b, R = [], [], []
    for w in range(W + 1):
        if w == 0:
            lo, hi = start.copy(), start.copy()
        elif w == W:
            lo, hi = goal.copy(), goal.copy()
        else:
            lo = np.maximum(g[w] - r, lim_lo)
            hi = np.minimum(g[w] + r, lim_hi)
        shape = tuple(int(h - l + 1) for l, h in zip(lo, hi))
        cand = _box_poses(lo, hi)
        valid, _ = poses(arm, occ, cand)
        valid = valid.reshape(shape)
        if w == 0:
            reach_w = valid
        else:
            # exists q' in R_{w-1} with |q - q'|_inf <= delta: embed R_{w-1} in the
            # union frame, binary max filter of width 2*delta+1, cut out box w.
            plo, phi = lo_b[-1], hi_b[-1]
            ulo = np.minimum(plo, lo) - delta
            uhi = np.maximum(phi, hi) + delta
            frame = np.zeros(tuple(int(v) for v in (uhi - ulo + 1)), bool)
            sl = tuple(slice(int(a - u), int(b - u + 1)) for a, b, u in zip(plo, phi, ulo))
            frame[sl] = R[-1]
            dil = ndimage.maximum_filter(frame, size=2 * delta + 1, mode="constant", cval=False)
            sl2 = tuple(slice(int(a - u), int(b - u + 1)) for a, b, u in zip(lo, hi, ulo))
            reach_w = dil[sl2] & valid
        lo_b.append(lo)
        hi_b.append(hi)
        R.append(reach_w)
    if not R[W].any():
        return None
    path = np.zeros((W + 1, dof), np.int64)
    path[W] = goal
    for w in range(W, 0, -1):
        q = path[w]
        plo, phi = lo_b[w - 1], hi_b[w - 1]
        clo = np.maximum(plo, q - delta)
        chi = np.minimum(phi, q + delta)
        cand = _box_poses(clo, chi).astype(np.int64)
        idx = tuple((cand[:, k] - plo[k]) for k in range(dof))
        ok = R[w - 1][idx]
        cand = cand[ok]
        assert cand.shape[0] > 0
        l1 = np.abs(cand - g[w - 1]).sum(axis=1)
        keys = [cand[:, k] for k in range(dof - 1, -1, -1)] + [l1]
        pick = np.lexsort(keys)[0]
        path[w - 1] = cand[pick]
    return path.astype(np.int32)


def plan_path(arm, occ, start, target, W: int, delta: int, r0: int = 1, r1: int = 2, retries: int = 4,
              m: Optional[int] = None, approach=None):
    """Reach pose + path.  The reach search runs with every joint limited to
    start +- W*delta and the canonical order centred on the start pose; then the
    tube search from each of the first ``retries`` reach poses with tube radius r0,
    then r1 (adaptive relaxation after a failure, "Filtering for smoothness";
    another reach pose from the survivor set, Step 3).
    Returns (status, path[(W+1), dof] or None, reach result)."""
    start = np.asarray(start, np.int64)
    lim_lo, lim_hi = arm_limits(arm)
    if np.any(start < lim_lo) or np.any(start > lim_hi) or W < 0 or delta < 0:
        return E_ARG, None, None
    valid, _ = poses(arm, occ, start[None, :])
    if not valid[0]:
        return E_ARG, None, None
    wlo = np.maximum(lim_lo, start - W * delta)
    whi = np.minimum(lim_hi, start + W * delta)
    res = reach(arm, occ, target, m=m, want=retries, lo=wlo, hi=whi, ref=start, keep_sets=False,
                approach=approach)
    if res.status != OK:
        return NO_REACH, None, res
    for q in res.sols:
        radii = [r0] if r1 == r0 else [r0, r1]
        for r in radii:
            if W == 0:
                return OK, start[None, :].astype(np.int32), res
            p = tube_search(arm, occ, start, q, W, delta, r, lim_lo, lim_hi)
            if p is not None:
                return OK, p, res
    return NO_PATH, None, res


def replan_path(arm, occ, start, target, W: int, delta: int, ref_path, r0: int = 1, r1: int = 2,
                retries: int = 4, m: Optional[int] = None, approach=None):
    """Midcourse replanning ("Dynamic Obstacles"): among the paths of the first
    ``retries`` reach poses (each with tube radius r0, then r1, as in plan_path), the
    one whose mean distance to the original path ``ref_path`` [(W+1), dof] is smallest:
    the sum over the W+1 waypoints of the L1 joint distance in steps; ties by the earlier
    reach pose.  Returns (status, path or None, reach result)."""
    start = np.asarray(start, np.int64)
    ref_path = np.asarray(ref_path, np.int64).reshape(W + 1, -1)
    lim_lo, lim_hi = arm_limits(arm)
    if np.any(start < lim_lo) or np.any(start > lim_hi) or W < 0 or delta < 0:
        return E_ARG, None, None
    valid, _ = poses(arm, occ, start[None, :])
    if not valid[0]:
        return E_ARG, None, None
    wlo = np.maximum(lim_lo, start - W * delta)
    whi = np.minimum(lim_hi, start + W * delta)
    res = reach(arm, occ, target, m=m, want=retries, lo=wlo, hi=whi, ref=start, keep_sets=False,
                approach=approach)
    if res.status != OK:
        return NO_REACH, None, res
    best, best_cost = None, None
    for q in res.sols:
        radii = [r0] if r1 == r0 else [r0, r1]
        for r in radii:
            p = start[None, :].astype(np.int32) if W == 0 else tube_search(arm, occ, start, q, W, delta, r,
                                                                            lim_lo, lim_hi)
            if p is not None:
                cost = int(np.abs(np.asarray(p, np.int64) - ref_path).sum())
                if best_cost is None or cost < best_cost:
                    best, best_cost = p, cost
                break
    if best is None:
        return NO_PATH, None, res
    return OK, best, res


def arm_limits(arm):
    step = arm.step_cdeg
    lo = np.array(arm.lo_cdeg, np.int64) // step
    hi = np.array(arm.hi_cdeg, np.int64) // step
    return lo, hi


def key_fields(keys: np.ndarray, n: int):
    """Split state keys into (x, y, z, ia, ie) arrays."""
    keys = np.asarray(keys, np.uint64)
    ie = (keys & np.uint64(0xff)).astype(np.int64)
    ia = ((keys >> np.uint64(8)) & np.uint64(0xff)).astype(np.int64)
    v = (keys >> np.uint64(16)).astype(np.int64)
    return v % n, (v // n) % n, v // (n * n), ia, ie


# --------------------------------------------------------------------------
# Exact end point for a discrete pose ("Exact IK solution with discretized segment
# mappings").  Plain FP64 with the math module, one pose at a time.
# --------------------------------------------------------------------------

YAW = 0


def _unit(az_deg: float, el_deg: float) -> np.ndarray:
    """Direction of a segment at global azimuth / elevation (degrees)."""
    a, e = np.radians(az_deg), np.radians(el_deg)
    return np.array([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)])


def _wrap180(x: float) -> float:
    """x modulo 360 in (-180, 180]."""
    y = x % 360.0
    return y - 360.0 if y > 180.0 else y


def _angles_near(s: np.ndarray, ref_az: float, ref_el: float) -> Tuple[float, float]:
    """(az, el) of vector s, of its two names on the (az, el) torus -- (az, el) and
    (az + 180, 180 - el) point the same way -- the one nearer (ref_az, ref_el), unwrapped
    next to it.  A vertical s keeps ref_az."""
    L = float(np.linalg.norm(s))
    el = float(np.degrees(np.arcsin(np.clip(s[2] / L, -1.0, 1.0))))
    if np.hypot(s[0], s[1]) <= 1e-12 * L:
        az = ref_az
    else:
        az = float(np.degrees(np.arctan2(s[1], s[0])))
    best = None
    for a, e in ((az, el), (az + 180.0, 180.0 - el)):
        da, de = _wrap180(a - ref_az), _wrap180(e - ref_el)
        cost = abs(da) + abs(de)
        if best is None or cost < best[0]:
            best = (cost, ref_az + da, ref_el + de)
    return best[1], best[2]


def refine_ok_arm(arm) -> bool:
    """The last two segments each have two DOF: joints dof-4..dof-1 are a zero-length
    link, a link of the other kind, a zero-length link, a link of the other kind."""
    n = len(arm.types)
    if n < 4:
        return False
    t, L = list(arm.types), list(arm.lens)
    return (L[n - 4] == 0 and L[n - 2] == 0 and t[n - 4] != t[n - 3] and t[n - 2] != t[n - 1]
            and L[n - 3] > 0 and L[n - 1] > 0)


def refine(arm, q: Sequence[int], target: Sequence[float]) -> Tuple[int, np.ndarray]:
    """(status, joint angles in degrees).  The first dof-4 joints keep their discrete
    angles; the last two segments are recomputed so that the chain ends on `target`:
    P = end of the fixed part (continuous FK), Jd = the discrete pose's joint between
    the last two segments, J = the point at distance L3 from P and L4 from the target in
    the plane (P, target, Jd) on Jd's side; status 1 (discrete angles returned) when no
    such triangle exists."""
    n = len(arm.types)
    assert refine_ok_arm(arm)
    step = arm.step_cdeg / 100.0
    az, el = arm.az0_cdeg / 100.0, arm.el0_cdeg / 100.0
    dirs = []
    for k in range(n):
        if arm.types[k] == YAW:
            az += q[k] * step
        else:
            el += q[k] * step
        dirs.append((az, el))
    disc = np.array([q[k] * step for k in range(n)], dtype=np.float64)
    P = np.array(arm.base, dtype=np.float64)
    for k in range(n - 4):
        P = P + arm.lens[k] * _unit(*dirs[k])
    L3, L4 = float(arm.lens[n - 3]), float(arm.lens[n - 1])
    Jd = P + L3 * _unit(*dirs[n - 3])
    T = np.asarray(target, dtype=np.float64)
    v = T - P
    d = float(np.linalg.norm(v))
    if d == 0.0 or d > L3 + L4 or d < abs(L3 - L4):
        return NO_REACH, disc
    u = v / d
    a = (L3 * L3 - L4 * L4 + d * d) / (2.0 * d)
    h = float(np.sqrt(max(L3 * L3 - a * a, 0.0)))
    rel = Jd - P
    w = rel - np.dot(rel, u) * u
    if np.linalg.norm(w) <= 1e-9 * L3:
        i = int(np.argmin(np.abs(u)))
        e = np.zeros(3)
        e[i] = 1.0
        w = np.cross(u, e)
    w = w / np.linalg.norm(w)
    J = P + a * u + h * w
    az3, el3 = _angles_near(J - P, *dirs[n - 3])
    az4, el4 = _angles_near(T - J, *dirs[n - 1])
    prev = dirs[n - 5] if n >= 5 else (arm.az0_cdeg / 100.0, arm.el0_cdeg / 100.0)
    out = disc.copy()
    for k0, (pa, pe), (na_, ne) in ((n - 4, prev, (az3, el3)), (n - 2, (az3, el3), (az4, el4))):
        for k in (k0, k0 + 1):
            out[k] = (na_ - pa) if arm.types[k] == YAW else (ne - pe)
    return OK, out
