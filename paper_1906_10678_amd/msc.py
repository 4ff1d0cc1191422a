"""ctypes binding of libmsc (include/msc.h).

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  PyTorch provides the device workspace, the occupancy-grid buffers and the
stream.  Joint values are integer steps in this Python API and centidegrees at the
C boundary.  Importing works without a GPU; creating a Solver needs the built
library and a GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsc.so")

MAX_DOF = 16
OK, NO_REACH, NO_PATH = 0, 1, 2
E_ARG, E_NOMEM, E_HIP, E_CAPACITY, E_STATE = -1, -2, -3, -4, -5
CAPTURE_SETS, NO_PRUNE, PROFILE, FUSED_TRACK, COUNT_SETS = 1, 2, 4, 8, 16
KERNELS = ["fill", "tables", "raster", "orient", "seed", "expand_fwd", "expand_bwd", "compact", "join", "dmark",
           "dfs", "pose", "tube_valid", "tube_solve", "refine", "track"]
SET_F, SET_B, SET_C, SET_D = 0, 1, 2, 3

EXPORTS = [
    "msc_opts_default", "msc_ctx_create", "msc_ctx_destroy", "msc_scene_bytes", "msc_scene_create",
    "msc_scene_destroy", "msc_reach", "msc_path", "msc_pose_check", "msc_get_stats",
    "msc_debug_tables", "msc_debug_raster", "msc_debug_set", "msc_last_error", "msc_get_timings",
    "msc_ctx_set_lanes", "msc_lane_bytes", "msc_batch", "msc_query_bytes", "msc_server_start",
    "msc_server_submit", "msc_server_poll", "msc_server_wait", "msc_server_stop", "msc_refine", "msc_replan",
    "msc_scene_bytes_dynamic", "msc_scene_set_dynamic", "msc_server_step", "msc_server_take_replans",
    "msc_refine_static", "msc_refine_static_max", "msc_track_default", "msc_guided_path", "msc_pose_path",
    "msc_autotune", "msc_tune_load", "msc_tune_entries", "msc_short_path", "msc_gms_quiver", "msc_gms_reach", "msc_gms_reach_first", "msc_server_set_limit",
]


class MscArm(ctypes.Structure):
    _fields_ = [("dof", ctypes.c_int32), ("step_cdeg", ctypes.c_int32), ("samples", ctypes.c_int32),
                ("base", ctypes.c_int32 * 3), ("az0_cdeg", ctypes.c_int32), ("el0_cdeg", ctypes.c_int32),
                ("type", ctypes.c_int32 * MAX_DOF), ("len_vox", ctypes.c_int32 * MAX_DOF),
                ("lo_cdeg", ctypes.c_int32 * MAX_DOF), ("hi_cdeg", ctypes.c_int32 * MAX_DOF)]


class MscTrack(ctypes.Structure):
    _fields_ = [("tracked", ctypes.c_int32), ("max_delta_cdeg", ctypes.c_int32),
                ("relaxed_delta_cdeg", ctypes.c_int32), ("eps2_vox", ctypes.c_int32)]


class MscGmsArm(ctypes.Structure):
    _fields_ = [("len", ctypes.c_double * 4), ("base", ctypes.c_int32 * 3), ("step_cdeg", ctypes.c_int32),
                ("min_ring", ctypes.c_int32), ("samples", ctypes.c_int32), ("seg1_min_el_cdeg", ctypes.c_int32),
                ("max_flex_cdeg", ctypes.c_int32 * 3), ("approach_az_cdeg", ctypes.c_int32),
                ("approach_el_cdeg", ctypes.c_int32), ("approach_half_cdeg", ctypes.c_int32), ("eps", ctypes.c_double)]


def make_gms_arm(arm) -> MscGmsArm:
    """From an object with lens, base, step_cdeg, m_min, samples, seg1_min_el_cdeg,
    max_flex_cdeg, approach (None or (az, el, half) cdeg) and eps."""
    a = MscGmsArm()
    for k in range(4):
        a.len[k] = float(arm.lens[k])
    for i in range(3):
        a.base[i] = int(arm.base[i])
        a.max_flex_cdeg[i] = int(arm.max_flex_cdeg[i])
    a.step_cdeg, a.min_ring, a.samples = arm.step_cdeg, arm.m_min, arm.samples
    a.seg1_min_el_cdeg = arm.seg1_min_el_cdeg
    ap = arm.approach
    a.approach_az_cdeg, a.approach_el_cdeg, a.approach_half_cdeg = (0, 0, -1) if ap is None else tuple(int(v) for v in ap)
    a.eps = float(arm.eps)
    return a


def gms_quiver(step_cdeg: int, min_ring: int = 4) -> np.ndarray:
    """The library's quiver (host code, no GPU needed): (count, 3) FP64."""
    L = load_library()
    n = L.msc_gms_quiver(step_cdeg, min_ring, None, 0)
    out = np.zeros((max(n, 1), 3), np.float64)
    L.msc_gms_quiver(step_cdeg, min_ring, _ptr(out, ctypes.c_double), n)
    return out[:n]


class MscBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("ext", ctypes.c_int32 * 3)]


class MscSphere(ctypes.Structure):
    _fields_ = [("c", ctypes.c_int32 * 3), ("r", ctypes.c_int32)]


def _struct_array(cls, rows: np.ndarray):
    """A ctypes array of `cls` (a struct of int32 fields only) holding the rows of an
    int32 array in field order (at least one element)."""
    rows = np.ascontiguousarray(rows, np.int32)
    assert rows.size * 4 == len(rows) * ctypes.sizeof(cls)
    out = (cls * max(1, len(rows)))()
    if len(rows):
        ctypes.memmove(out, rows.ctypes.data, rows.nbytes)
    return out


class MscTiming(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("stage", ctypes.c_int32), ("in_count", ctypes.c_int64),
                ("out_count", ctypes.c_int64), ("ms", ctypes.c_float), ("out_words", ctypes.c_int64)]


class MscQuery(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("arm", ctypes.POINTER(MscArm)), ("kind", ctypes.c_int32),
                ("target", ctypes.c_int32 * 3), ("start_cdeg", ctypes.POINTER(ctypes.c_int32)),
                ("waypoints", ctypes.c_int32), ("max_delta_cdeg", ctypes.c_int32),
                ("out", ctypes.POINTER(ctypes.c_int32)), ("status", ctypes.c_int), ("latency_ms", ctypes.c_float),
                ("ref_cdeg", ctypes.POINTER(ctypes.c_int32)), ("tick", ctypes.c_int64),
                ("execute_ticks", ctypes.c_int32), ("replan_depth", ctypes.c_int32), ("error", ctypes.c_char * 128),
                ("virtual_arm", ctypes.POINTER(MscArm)), ("track", MscTrack), ("rows", ctypes.c_int32)]


class MscStepReport(ctypes.Structure):
    _fields_ = [("executing", ctypes.c_int32), ("finished", ctypes.c_int32), ("stopped", ctypes.c_int32),
                ("replans", ctypes.c_int32), ("poses_checked", ctypes.c_int64)]


class MscOpts(ctypes.Structure):
    _fields_ = [("split_m", ctypes.c_int32), ("tube_r0", ctypes.c_int32), ("tube_r1", ctypes.c_int32),
                ("reach_retries", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("approach_az_cdeg", ctypes.c_int32), ("approach_el_cdeg", ctypes.c_int32),
                ("approach_half_cdeg", ctypes.c_int32)]


class MscStats(ctypes.Structure):
    _fields_ = [("split_m", ctypes.c_int32), ("dof", ctypes.c_int32),
                ("fwd_count", ctypes.c_int64 * (MAX_DOF + 1)), ("bwd_count", ctypes.c_int64 * (MAX_DOF + 1)),
                ("join_count", ctypes.c_int64),
                ("fwd_dense", ctypes.c_int32 * (MAX_DOF + 1)), ("bwd_dense", ctypes.c_int32 * (MAX_DOF + 1)),
                ("attempts", ctypes.c_int32), ("tube_r", ctypes.c_int32), ("reach_index", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmsc.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmsc.so is not built (%s); run paper_1906_10678_amd/build.py" % path)
    L = ctypes.CDLL(path)
    P, c_void_p = ctypes.POINTER, ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    L.msc_opts_default.argtypes = [P(MscOpts)]
    L.msc_opts_default.restype = None
    L.msc_ctx_create.argtypes = [ctypes.c_int, c_void_p, c_void_p, u64, P(c_void_p)]
    L.msc_ctx_destroy.argtypes = [c_void_p]
    L.msc_scene_bytes.argtypes = [i32]
    L.msc_scene_bytes.restype = u64
    L.msc_scene_create.argtypes = [c_void_p, i32, i32, P(MscBox), i32, P(MscSphere), i32, c_void_p, u64,
                                   P(c_void_p)]
    L.msc_scene_destroy.argtypes = [c_void_p]
    L.msc_reach.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), P(MscOpts), P(i32)]
    L.msc_path.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), P(i32), i32, i32, P(MscOpts), P(i32)]
    L.msc_pose_check.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), i64, P(ctypes.c_uint8), P(i32)]
    L.msc_replan.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), P(i32), i32, i32, P(i32), P(MscOpts), P(i32)]
    L.msc_get_stats.argtypes = [c_void_p, P(MscStats)]
    L.msc_refine.argtypes = [c_void_p, P(MscArm), P(i32), P(ctypes.c_double), i64, P(ctypes.c_double), P(i32)]
    L.msc_track_default.argtypes = [P(MscTrack)]
    L.msc_track_default.restype = None
    L.msc_guided_path.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), P(MscTrack), P(MscOpts), P(i32), P(i32)]
    L.msc_pose_path.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), P(i32), P(MscArm), P(MscTrack), P(MscOpts),
                                P(i32), P(i32)]
    L.msc_short_path.argtypes = [c_void_p, c_void_p, P(MscArm), P(i32), i32, i32, P(MscTrack), P(MscOpts), P(i32),
                                 P(i32), P(i32)]
    L.msc_server_set_limit.argtypes = [c_void_p, i32]
    L.msc_gms_quiver.argtypes = [i32, i32, P(ctypes.c_double), i32]
    L.msc_gms_quiver.restype = i32
    L.msc_gms_reach.argtypes = [c_void_p, c_void_p, P(MscGmsArm), P(i32), i32, P(i64), P(i32), P(ctypes.c_double),
                                P(i32)]
    L.msc_gms_reach_first.argtypes = [c_void_p, c_void_p, P(MscGmsArm), P(i32), i32, P(i64), P(i32),
                                      P(ctypes.c_double), P(i32)]
    L.msc_autotune.argtypes = [c_void_p, P(MscQuery), i32, P(MscOpts), ctypes.c_char_p]
    L.msc_tune_load.argtypes = [c_void_p, ctypes.c_char_p]
    L.msc_tune_entries.argtypes = [c_void_p, P(i32), i32, P(i32)]
    L.msc_refine_static.argtypes = L.msc_refine.argtypes
    L.msc_refine_static_max.argtypes = [i32]
    L.msc_refine_static_max.restype = i64
    L.msc_debug_tables.argtypes = [c_void_p, P(MscArm), i32, P(i32), P(i32)]
    L.msc_debug_raster.argtypes = [c_void_p, c_void_p, P(ctypes.c_uint8)]
    L.msc_debug_set.argtypes = [c_void_p, i32, i32, P(u64), u64, P(u64)]
    L.msc_get_timings.argtypes = [c_void_p, P(MscTiming), i32, P(i32)]
    L.msc_ctx_set_lanes.argtypes = [c_void_p, i32]
    L.msc_lane_bytes.argtypes = [c_void_p]
    L.msc_lane_bytes.restype = u64
    L.msc_batch.argtypes = [c_void_p, P(MscQuery), i32, P(MscOpts)]
    L.msc_query_bytes.argtypes = [P(MscQuery)]
    L.msc_query_bytes.restype = u64
    L.msc_server_start.argtypes = [c_void_p, P(MscOpts)]
    L.msc_server_submit.argtypes = [c_void_p, P(MscQuery), P(u64)]
    L.msc_server_poll.argtypes = [c_void_p, u64, P(i32)]
    L.msc_server_wait.argtypes = [c_void_p, u64]
    L.msc_server_stop.argtypes = [c_void_p]
    L.msc_scene_bytes_dynamic.argtypes = [i32, i32]
    L.msc_scene_bytes_dynamic.restype = u64
    L.msc_scene_set_dynamic.argtypes = [c_void_p, P(MscBox), i32, i64]
    L.msc_server_step.argtypes = [c_void_p, i64, P(MscStepReport)]
    L.msc_server_take_replans.argtypes = [c_void_p, P(MscQuery), i32, P(i32)]
    L.msc_last_error.argtypes = [c_void_p]
    L.msc_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("msc_opts_default", "msc_scene_bytes", "msc_last_error", "msc_lane_bytes",
                        "msc_query_bytes", "msc_scene_bytes_dynamic", "msc_refine_static_max",
                        "msc_track_default", "msc_gms_quiver"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def make_arm(arm) -> MscArm:
    """msc_arm from a duck-typed arm (types, lens, lo_cdeg, hi_cdeg, step_cdeg, base,
    samples, az0_cdeg, el0_cdeg)."""
    a = MscArm()
    n = len(arm.types)
    a.dof = n
    a.step_cdeg = int(arm.step_cdeg)
    a.samples = int(arm.samples)
    for i in range(3):
        a.base[i] = int(arm.base[i])
    a.az0_cdeg = int(arm.az0_cdeg)
    a.el0_cdeg = int(arm.el0_cdeg)
    for k in range(n):
        a.type[k] = int(arm.types[k])
        a.len_vox[k] = int(arm.lens[k])
        a.lo_cdeg[k] = int(arm.lo_cdeg[k])
        a.hi_cdeg[k] = int(arm.hi_cdeg[k])
    return a


def make_opts(split_m: int = -1, tube_r0: int = 1, tube_r1: int = 2, retries: int = 4, flags: int = 0,
              approach=None) -> MscOpts:
    """approach: None, or (az_cdeg, el_cdeg, half_cdeg) of the last segment's approach cone."""
    o = MscOpts()
    o.split_m, o.tube_r0, o.tube_r1, o.reach_retries, o.flags = split_m, tube_r0, tube_r1, retries, flags
    o.approach_az_cdeg, o.approach_el_cdeg, o.approach_half_cdeg = (0, 0, -1) if approach is None else approach
    return o


def make_track(a: "MscArm", tracked: int = -1, delta: int = -1, delta2: int = -1, eps2: int = 9) -> "MscTrack":
    """delta / delta2 in steps (-1: the library's defaults)."""
    t = MscTrack()
    t.tracked = tracked
    t.max_delta_cdeg = -1 if delta < 0 else delta * a.step_cdeg
    t.relaxed_delta_cdeg = -1 if delta2 < 0 else delta2 * a.step_cdeg
    t.eps2_vox = eps2
    return t


class QuerySpec:
    """A query for msc_batch / the server: reach (kind 0), reach + path (kind 1),
    reach-pose-guided path (kind 2) or path between poses through a virtual arm (kind 3);
    owns the ctypes buffers until the query completes.  track = (tracked, delta, delta2,
    eps2) with deltas in steps (-1: defaults)."""

    def __init__(self, scene: "Scene", arm, target, start=None, waypoints: int = 0, delta: int = 0, ref=None,
                 execute_ticks: int = 0, kind: Optional[int] = None, virtual_arm=None, track=(-1, -1, -1, 9)):
        self.scene = scene
        self.arm_c = make_arm(arm)
        self.dof = self.arm_c.dof
        self.step = self.arm_c.step_cdeg
        self.kind = (0 if start is None else 1) if kind is None else int(kind)
        self.waypoints = int(waypoints)
        self.varm_c = make_arm(virtual_arm) if virtual_arm is not None else None
        if self.kind == 1:
            rows = self.waypoints + 1
        elif self.kind == 2:
            k = self.dof - 2 if track[0] < 0 else track[0]
            rows = self.arm_c.samples * max(k - 1, 0) + 1
        elif self.kind == 3:
            rows = self.varm_c.samples * self.varm_c.dof + 1
        else:
            rows = 1
        self.out = np.zeros(rows * self.dof, np.int32)
        self.start = None if start is None else np.ascontiguousarray(np.asarray(start, np.int32) * self.step)
        q = MscQuery()
        q.scene = scene.handle
        q.arm = ctypes.pointer(self.arm_c)
        q.kind = self.kind
        for i in range(3):
            q.target[i] = int(target[i])
        q.start_cdeg = _ptr(self.start, ctypes.c_int32) if self.start is not None else None
        q.waypoints = self.waypoints
        q.max_delta_cdeg = int(delta) * self.step
        q.out = _ptr(self.out, ctypes.c_int32)
        # replanning: the original path's rows (steps), kept alive with the query
        self.ref = None if ref is None else np.ascontiguousarray(
            np.asarray(ref, np.int32).reshape(self.waypoints + 1, self.dof) * self.step)
        q.ref_cdeg = _ptr(self.ref, ctypes.c_int32) if self.ref is not None else None
        q.execute_ticks = int(execute_ticks)
        q.virtual_arm = ctypes.pointer(self.varm_c) if self.varm_c is not None else None
        q.track = make_track(self.arm_c, *track)
        q.status = -100
        self.c = q

    @property
    def tick(self) -> int:
        """The logical tick of the scene grid the query was solved on."""
        return int(self.c.tick)

    @property
    def error(self) -> str:
        return self.c.error.decode()

    def result(self):
        """(status, joint values in steps: [dof] for reach, [(W+1), dof] for path, latency ms)."""
        st = self.c.status
        if st != OK:
            return st, None, self.c.latency_ms
        v = self.out // self.step
        if self.kind == 0:
            return st, v, self.c.latency_ms
        if self.kind == 1:
            return st, v.reshape(self.waypoints + 1, self.dof), self.c.latency_ms
        r = self.c.rows
        return st, v[:r * self.dof].reshape(r, self.dof), self.c.latency_ms


class MscError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("msc status %d: %s" % (status, message))
        self.status = status


class Scene:
    def __init__(self, solver: "Solver", handle, grid_tensor, n: int):
        self.solver = solver
        self.handle = handle
        self.grid = grid_tensor
        self.n = n

    def close(self):
        if self.handle:
            self.solver.lib.msc_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One library context on one GPU with a torch-owned device workspace."""

    def __init__(self, device: int = 0, workspace_bytes: int = 8 << 30, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the solver runs only on the HIP device")
        self.lib = load_library()
        self.torch = torch
        self.device = device
        self.dev = torch.device("cuda", device)
        self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        h = ctypes.c_void_p()
        rc = self.lib.msc_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.c_void_p(self.workspace.data_ptr()), int(workspace_bytes),
                                     ctypes.byref(h))
        if rc != OK:
            raise MscError(rc, "msc_ctx_create failed")
        self.ctx = h

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.msc_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return self.lib.msc_last_error(self.ctx).decode()

    def _check(self, rc: int, what: str) -> int:
        if rc < 0:
            raise MscError(rc, "%s: %s" % (what, self.error()))
        return rc

    # -- scenes -------------------------------------------------------------
    def scene(self, sc, ticks: int = 0) -> Scene:
        """A scene's grid on the device; ticks > 0 leaves room for that many grids of
        logical ticks with moving obstacles (set_dynamic)."""
        n = int(sc.n)
        nbytes = int(self.lib.msc_scene_bytes_dynamic(n, ticks) if ticks > 0 else self.lib.msc_scene_bytes(n))
        if nbytes == 0:
            raise MscError(E_ARG, "bad grid size or tick count")
        grid = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.dev)
        boxes = np.asarray(sc.boxes, np.int32).reshape(-1, 6)
        sph = np.asarray(sc.spheres, np.int32).reshape(-1, 4)
        B = _struct_array(MscBox, boxes)
        S = _struct_array(MscSphere, sph)
        h = ctypes.c_void_p()
        rc = self.lib.msc_scene_create(self.ctx, n, int(sc.dilate), B, len(boxes), S, len(sph),
                                       ctypes.c_void_p(grid.data_ptr()), nbytes, ctypes.byref(h))
        self._check(rc, "msc_scene_create")
        return Scene(self, h, grid, n)

    def set_dynamic(self, scene: Scene, boxes, tick: int):
        """msc_scene_set_dynamic: the scene's grid of `tick` = static obstacles + boxes
        (k, 6) int (lo x, y, z, extent x, y, z), dilated like the static ones."""
        boxes = np.asarray(boxes, np.int32).reshape(-1, 6)
        B = _struct_array(MscBox, boxes)
        self._check(self.lib.msc_scene_set_dynamic(scene.handle, B, len(boxes), int(tick)), "msc_scene_set_dynamic")

    # -- solving ------------------------------------------------------------
    def reach(self, scene: Scene, arm, target: Sequence[int], split_m: int = -1,
              flags: int = 0, approach=None) -> Tuple[int, Optional[np.ndarray]]:
        a = make_arm(arm)
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        out = np.zeros(a.dof, np.int32)
        o = make_opts(split_m=split_m, flags=flags, approach=approach)
        rc = self.lib.msc_reach(self.ctx, scene.handle, ctypes.byref(a), _ptr(t, ctypes.c_int32), ctypes.byref(o),
                                _ptr(out, ctypes.c_int32))
        self._check(rc, "msc_reach")
        return rc, (out // a.step_cdeg if rc == OK else None)

    def path(self, scene: Scene, arm, start: Sequence[int], target: Sequence[int], waypoints: int, delta: int,
             split_m: int = -1, tube_r0: int = 1, tube_r1: int = 2, retries: int = 4,
             flags: int = 0, approach=None) -> Tuple[int, Optional[np.ndarray]]:
        a = make_arm(arm)
        s = np.ascontiguousarray(np.asarray(start, np.int32) * a.step_cdeg)
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        out = np.zeros((waypoints + 1) * a.dof, np.int32)
        o = make_opts(split_m, tube_r0, tube_r1, retries, flags, approach)
        rc = self.lib.msc_path(self.ctx, scene.handle, ctypes.byref(a), _ptr(s, ctypes.c_int32),
                               _ptr(t, ctypes.c_int32), int(waypoints), int(delta) * a.step_cdeg, ctypes.byref(o),
                               _ptr(out, ctypes.c_int32))
        self._check(rc, "msc_path")
        return rc, (out.reshape(waypoints + 1, a.dof) // a.step_cdeg if rc == OK else None)

    def guided_path(self, scene: Scene, arm, target: Sequence[int], tracked: int = -1, delta: int = -1,
                    delta2: int = -1, eps2: int = 9, split_m: int = -1, retries: int = 4, flags: int = 0,
                    approach=None) -> Tuple[int, Optional[np.ndarray]]:
        """msc_guided_path: (status, rows[(M+1), dof] in steps, root waypoint pose first).
        delta / delta2 in steps (-1: one and two steps)."""
        a = make_arm(arm)
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        tr = make_track(a, tracked, delta, delta2, eps2)
        k = a.dof - 2 if tracked < 0 else tracked
        out = np.zeros((a.samples * max(k - 1, 0) + 1) * a.dof, np.int32)
        rows = ctypes.c_int32()
        o = make_opts(split_m, 1, 2, retries, flags, approach)
        rc = self.lib.msc_guided_path(self.ctx, scene.handle, ctypes.byref(a), _ptr(t, ctypes.c_int32),
                                      ctypes.byref(tr), ctypes.byref(o), _ptr(out, ctypes.c_int32), ctypes.byref(rows))
        self._check(rc, "msc_guided_path")
        if rc != OK:
            return rc, None
        return rc, out[:rows.value * a.dof].reshape(rows.value, a.dof) // a.step_cdeg

    def short_path(self, scene: Scene, arm, target: Sequence[int], rho2: int = 4, segments: int = -1,
                   tracked: int = -1, delta: int = -1, delta2: int = -1, eps2: int = 9, split_m: int = -1,
                   retries: int = 4, flags: int = 0):
        """msc_short_path: (status, rows[(M+1), dof] in steps or None, hit or None) with hit =
        dict(k, s, length, q[k] in steps); segments -1: min(4, dof - 1)."""
        a = make_arm(arm)
        K = min(4, a.dof - 1) if segments < 0 else segments
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        tr = make_track(a, tracked, delta, delta2, eps2)
        k2 = a.dof - 2 if tracked < 0 else tracked
        out = np.zeros((a.samples * max(K - 1, k2 - 1) + 2) * a.dof, np.int32)
        rows = ctypes.c_int32()
        hit = np.zeros(MAX_DOF + 3, np.int32)
        o = make_opts(split_m, 1, 2, retries, flags)
        rc = self.lib.msc_short_path(self.ctx, scene.handle, ctypes.byref(a), _ptr(t, ctypes.c_int32), int(rho2), K,
                                     ctypes.byref(tr), ctypes.byref(o), _ptr(out, ctypes.c_int32), ctypes.byref(rows),
                                     _ptr(hit, ctypes.c_int32))
        self._check(rc, "msc_short_path")
        h = None
        if hit[0] > 0:
            h = {"k": int(hit[0]), "s": int(hit[1]), "length": int(hit[2]),
                 "q": hit[3:3 + hit[0]] // a.step_cdeg}
        if rc != OK:
            return rc, None, h
        return rc, out[:rows.value * a.dof].reshape(rows.value, a.dof) // a.step_cdeg, h

    def gms_reach(self, scene: Scene, arm, target: Sequence[int], want: int = 1, first_only: bool = False):
        """msc_gms_reach (msc_gms_reach_first with first_only): (status, solutions counted,
        sols[n, 3] (i, j, l), vectors[n, 6, 3])."""
        a = make_gms_arm(arm)
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        cnt = ctypes.c_int64()
        nsol = ctypes.c_int32()
        sols = np.zeros(want * 3, np.int32)
        vec = np.zeros(want * 18, np.float64)
        fn = self.lib.msc_gms_reach_first if first_only else self.lib.msc_gms_reach
        rc = fn(self.ctx, scene.handle, ctypes.byref(a), _ptr(t, ctypes.c_int32), int(want), ctypes.byref(cnt),
                _ptr(sols, ctypes.c_int32), _ptr(vec, ctypes.c_double), ctypes.byref(nsol))
        self._check(rc, "msc_gms_reach_first" if first_only else "msc_gms_reach")
        n = nsol.value
        return rc, int(cnt.value), sols[:3 * n].reshape(n, 3), vec[:18 * n].reshape(n, 6, 3)

    def pose_path(self, scene: Scene, arm, start: Sequence[int], target: Sequence[int], virtual_arm,
                  tracked: int = -1, delta: int = -1, delta2: int = -1, eps2: int = 9, split_m: int = -1,
                  retries: int = 4, flags: int = 0) -> Tuple[int, Optional[np.ndarray]]:
        """msc_pose_path: (status, rows[(M+1), dof] in steps, row 0 = start)."""
        a = make_arm(arm)
        va = make_arm(virtual_arm)
        s = np.ascontiguousarray(np.asarray(start, np.int32) * a.step_cdeg)
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        tr = make_track(a, tracked, delta, delta2, eps2)
        out = np.zeros((va.samples * va.dof + 1) * a.dof, np.int32)
        rows = ctypes.c_int32()
        o = make_opts(split_m, 1, 2, retries, flags)
        rc = self.lib.msc_pose_path(self.ctx, scene.handle, ctypes.byref(a), _ptr(s, ctypes.c_int32),
                                    _ptr(t, ctypes.c_int32), ctypes.byref(va), ctypes.byref(tr), ctypes.byref(o),
                                    _ptr(out, ctypes.c_int32), ctypes.byref(rows))
        self._check(rc, "msc_pose_path")
        if rc != OK:
            return rc, None
        return rc, out[:rows.value * a.dof].reshape(rows.value, a.dof) // a.step_cdeg

    def replan(self, scene: Scene, arm, start: Sequence[int], target: Sequence[int], waypoints: int, delta: int,
               ref_path, split_m: int = -1, tube_r0: int = 1, tube_r1: int = 2, retries: int = 4,
               flags: int = 0, approach=None) -> Tuple[int, Optional[np.ndarray]]:
        """msc_replan: the path of the first `retries` reach poses nearest ref_path
        [(waypoints+1), dof] (steps)."""
        a = make_arm(arm)
        s = np.ascontiguousarray(np.asarray(start, np.int32) * a.step_cdeg)
        t = np.ascontiguousarray(np.asarray(target, np.int32))
        ref = np.ascontiguousarray(np.asarray(ref_path, np.int32).reshape(waypoints + 1, a.dof) * a.step_cdeg)
        out = np.zeros((waypoints + 1) * a.dof, np.int32)
        o = make_opts(split_m, tube_r0, tube_r1, retries, flags, approach)
        rc = self.lib.msc_replan(self.ctx, scene.handle, ctypes.byref(a), _ptr(s, ctypes.c_int32),
                                 _ptr(t, ctypes.c_int32), int(waypoints), int(delta) * a.step_cdeg,
                                 _ptr(ref, ctypes.c_int32), ctypes.byref(o), _ptr(out, ctypes.c_int32))
        self._check(rc, "msc_replan")
        return rc, (out.reshape(waypoints + 1, a.dof) // a.step_cdeg if rc == OK else None)

    def pose_check(self, scene: Scene, arm, q) -> Tuple[np.ndarray, np.ndarray]:
        a = make_arm(arm)
        q = np.ascontiguousarray(np.asarray(q, np.int32).reshape(-1, a.dof) * a.step_cdeg)
        valid = np.zeros(q.shape[0], np.uint8)
        ends = np.zeros((q.shape[0], 3), np.int32)
        rc = self.lib.msc_pose_check(self.ctx, scene.handle, ctypes.byref(a), _ptr(q, ctypes.c_int32), q.shape[0],
                                     _ptr(valid, ctypes.c_uint8), _ptr(ends, ctypes.c_int32))
        self._check(rc, "msc_pose_check")
        return valid.astype(bool), ends.astype(np.int64)

    def refine(self, arm, q, targets) -> Tuple[np.ndarray, np.ndarray]:
        """Exact end points (msc_refine): q[count, dof] in steps, targets[count, 3] (voxel
        units); returns (angles in degrees [count, dof], status [count])."""
        a = make_arm(arm)
        q = np.ascontiguousarray(np.asarray(q, np.int32).reshape(-1, a.dof) * a.step_cdeg)
        t = np.ascontiguousarray(np.asarray(targets, np.float64).reshape(-1, 3))
        if t.shape[0] != q.shape[0]:
            raise ValueError("one target per pose")
        ang = np.zeros(q.shape, np.float64)
        st = np.zeros(q.shape[0], np.int32)
        rc = self.lib.msc_refine(self.ctx, ctypes.byref(a), _ptr(q, ctypes.c_int32), _ptr(t, ctypes.c_double),
                                 q.shape[0], _ptr(ang, ctypes.c_double), _ptr(st, ctypes.c_int32))
        self._check(rc, "msc_refine")
        return ang, st

    def refine_static(self, arm, q, targets) -> Tuple[np.ndarray, np.ndarray]:
        """msc_refine_static: as refine(), with the device staging in the library's fixed
        buffer (no workspace use); at most msc_refine_static_max(dof) poses."""
        a = make_arm(arm)
        q = np.ascontiguousarray(np.asarray(q, np.int32).reshape(-1, a.dof) * a.step_cdeg)
        t = np.ascontiguousarray(np.asarray(targets, np.float64).reshape(-1, 3))
        if t.shape[0] != q.shape[0]:
            raise ValueError("one target per pose")
        ang = np.zeros(q.shape, np.float64)
        st = np.zeros(q.shape[0], np.int32)
        rc = self.lib.msc_refine_static(self.ctx, ctypes.byref(a), _ptr(q, ctypes.c_int32),
                                        _ptr(t, ctypes.c_double), q.shape[0], _ptr(ang, ctypes.c_double),
                                        _ptr(st, ctypes.c_int32))
        self._check(rc, "msc_refine_static")
        return ang, st

    def refine_static_max(self, dof: int) -> int:
        return int(self.lib.msc_refine_static_max(dof))

    def pose_fn_for(self, arm, sc):
        """A synth-compatible pose function backed by the GPU library."""
        scene = self.scene(sc)

        def f(q):
            return self.pose_check(scene, arm, q)

        f.scene = scene
        return f

    def stats(self) -> dict:
        s = MscStats()
        self._check(self.lib.msc_get_stats(self.ctx, ctypes.byref(s)), "msc_get_stats")
        n = s.dof
        return dict(split_m=s.split_m, dof=n, fwd_count=list(s.fwd_count[:n + 1]),
                    bwd_count=list(s.bwd_count[:n + 1]), join_count=s.join_count,
                    fwd_dense=list(s.fwd_dense[:n + 1]), bwd_dense=list(s.bwd_dense[:n + 1]),
                    attempts=s.attempts, tube_r=s.tube_r, reach_index=s.reach_index)

    def timings(self) -> list:
        """Launch records of the last call made with PROFILE: (kernel, stage, in, out, ms)."""
        cnt = ctypes.c_int32()
        self._check(self.lib.msc_get_timings(self.ctx, None, 0, ctypes.byref(cnt)), "msc_get_timings")
        buf = (MscTiming * max(1, cnt.value))()
        self._check(self.lib.msc_get_timings(self.ctx, buf, cnt.value, ctypes.byref(cnt)), "msc_get_timings")
        return [(KERNELS[t.kernel], t.stage, t.in_count, t.out_count, t.ms) for t in buf[:cnt.value]]

    def timing_words(self) -> list:
        """out_words of the last call's launch records (-1 where not counted)."""
        cnt = ctypes.c_int32()
        self._check(self.lib.msc_get_timings(self.ctx, None, 0, ctypes.byref(cnt)), "msc_get_timings")
        buf = (MscTiming * max(1, cnt.value))()
        self._check(self.lib.msc_get_timings(self.ctx, buf, cnt.value, ctypes.byref(cnt)), "msc_get_timings")
        return [int(t.out_words) for t in buf[:cnt.value]]

    # -- lanes, batches, server ----------------------------------------------
    def set_lanes(self, nworkers: int):
        self._check(self.lib.msc_ctx_set_lanes(self.ctx, int(nworkers)), "msc_ctx_set_lanes")

    def lane_bytes(self) -> int:
        return int(self.lib.msc_lane_bytes(self.ctx))

    def batch(self, specs, split_m: int = -1, flags: int = 0, approach=None, tube_r0: int = 1, tube_r1: int = 2,
              retries: int = 4):
        """Solve QuerySpecs with msc_batch; returns their results."""
        arr = (MscQuery * max(1, len(specs)))()
        for i, sp in enumerate(specs):
            arr[i] = sp.c
        o = make_opts(split_m, tube_r0, tube_r1, retries, flags, approach)
        self._check(self.lib.msc_batch(self.ctx, arr, len(specs), ctypes.byref(o)), "msc_batch")
        for i, sp in enumerate(specs):
            sp.c.status = arr[i].status
            sp.c.latency_ms = arr[i].latency_ms
            sp.c.tick = arr[i].tick
            sp.c.error = arr[i].error
            sp.c.rows = arr[i].rows
        return [sp.result() for sp in specs]

    def autotune(self, specs, cache_path: Optional[str] = None, split_m: int = -1, approach=None):
        """msc_autotune over QuerySpecs (solved on the context's own lane); returns the
        chosen entries (kernel name, size class, variant, grid cap, lanes change)."""
        arr = (MscQuery * max(1, len(specs)))()
        for i, sp in enumerate(specs):
            arr[i] = sp.c
        o = make_opts(split_m=split_m, approach=approach)
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.msc_autotune(self.ctx, arr, len(specs), ctypes.byref(o), path), "msc_autotune")
        return self.tune_entries()

    def tune_load(self, cache_path: str):
        self._check(self.lib.msc_tune_load(self.ctx, cache_path.encode()), "msc_tune_load")

    def tune_entries(self):
        cnt = ctypes.c_int32()
        self._check(self.lib.msc_tune_entries(self.ctx, None, 0, ctypes.byref(cnt)), "msc_tune_entries")
        buf = np.zeros(max(1, cnt.value) * 5, np.int32)
        self._check(self.lib.msc_tune_entries(self.ctx, _ptr(buf, ctypes.c_int32), cnt.value, ctypes.byref(cnt)),
                    "msc_tune_entries")
        return [(KERNELS[r[0]], int(r[1]), int(r[2]), int(r[3]), int(r[4])) for r in buf[:cnt.value * 5].reshape(-1, 5)]

    def query_bytes(self, spec: QuerySpec) -> int:
        return int(self.lib.msc_query_bytes(ctypes.byref(spec.c)))

    def server_start(self, split_m: int = -1, flags: int = 0, approach=None):
        o = make_opts(split_m=split_m, flags=flags, approach=approach)
        self._check(self.lib.msc_server_start(self.ctx, ctypes.byref(o)), "msc_server_start")
        self._inflight = {}

    def server_set_limit(self, max_pending: int):
        """msc_server_set_limit: refuse submissions while max_pending queries wait (0: none)."""
        self._check(self.lib.msc_server_set_limit(self.ctx, int(max_pending)), "msc_server_set_limit")

    def submit(self, spec: QuerySpec, shed: bool = False) -> Optional[int]:
        """msc_server_submit: the ticket; with shed, None when the server refuses the query
        for its queue depth (E_CAPACITY) instead of raising."""
        t = ctypes.c_uint64()
        rc = self.lib.msc_server_submit(self.ctx, ctypes.byref(spec.c), ctypes.byref(t))
        if shed and rc == E_CAPACITY:
            return None
        self._check(rc, "msc_server_submit")
        self._inflight[t.value] = spec
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        self._check(self.lib.msc_server_poll(self.ctx, ticket, ctypes.byref(d)), "msc_server_poll")
        if d.value:
            self._inflight.pop(ticket, None)
        return bool(d.value)

    def wait(self, ticket: int):
        self._check(self.lib.msc_server_wait(self.ctx, ticket), "msc_server_wait")
        return self._inflight.pop(ticket).result()

    def server_stop(self):
        self._check(self.lib.msc_server_stop(self.ctx), "msc_server_stop")

    def server_step(self, tick: int) -> dict:
        """msc_server_step: re-validate executing paths at `tick`, queue replans."""
        r = MscStepReport()
        self._check(self.lib.msc_server_step(self.ctx, int(tick), ctypes.byref(r)), "msc_server_step")
        return dict(executing=r.executing, finished=r.finished, stopped=r.stopped, replans=r.replans,
                    poses_checked=r.poses_checked)

    def take_replans(self) -> list:
        """Completed replans issued by server_step, as dicts (joint values in steps)."""
        if getattr(self, "_replan_buf", None) is None:
            self._replan_buf = (MscQuery * 256)()
        buf, cap = self._replan_buf, 256
        cnt = ctypes.c_int32()
        self._check(self.lib.msc_server_take_replans(self.ctx, buf, cap, ctypes.byref(cnt)), "msc_server_take_replans")
        out = []
        for q in buf[:cnt.value]:
            a = q.arm.contents
            n, step, W = a.dof, a.step_cdeg, q.waypoints
            rows = lambda p, k: np.ctypeslib.as_array(p, shape=(k * n,)).reshape(k, n) // step  # noqa: E731
            out.append(dict(status=q.status, tick=int(q.tick), latency_ms=float(q.latency_ms), depth=q.replan_depth,
                            scene=q.scene, dof=n, step=step, arm_types=list(a.type[:n]), arm_lens=list(a.len_vox[:n]),
                            lo_cdeg=list(a.lo_cdeg[:n]), hi_cdeg=list(a.hi_cdeg[:n]), base=tuple(a.base),
                            target=tuple(q.target), waypoints=W, delta=q.max_delta_cdeg // step,
                            start=rows(q.start_cdeg, 1)[0].copy(), ref=rows(q.ref_cdeg, W + 1).copy(),
                            path=rows(q.out, W + 1).copy() if q.status == OK else None,
                            error=q.error.decode()))
        return out

    # -- debug --------------------------------------------------------------
    def debug_tables(self, arm, stage: int):
        a = make_arm(arm)
        na = 36000 // a.step_cdeg
        off = np.zeros((na, na, 3), np.int32)
        sweep = np.zeros((na, na, a.samples, 3), np.int32)
        rc = self.lib.msc_debug_tables(self.ctx, ctypes.byref(a), stage, _ptr(off, ctypes.c_int32),
                                       _ptr(sweep, ctypes.c_int32))
        self._check(rc, "msc_debug_tables")
        return off, sweep

    def debug_raster(self, scene: Scene) -> np.ndarray:
        n = scene.n
        occ = np.zeros((n, n, n), np.uint8)
        self._check(self.lib.msc_debug_raster(self.ctx, scene.handle, _ptr(occ, ctypes.c_uint8)), "msc_debug_raster")
        return occ

    def debug_set(self, which: int, stage: int) -> np.ndarray:
        cnt = ctypes.c_uint64()
        self._check(self.lib.msc_debug_set(self.ctx, which, stage, None, 0, ctypes.byref(cnt)), "msc_debug_set")
        out = np.zeros(cnt.value, np.uint64)
        if cnt.value:
            self._check(self.lib.msc_debug_set(self.ctx, which, stage, _ptr(out, ctypes.c_uint64), cnt.value,
                                               ctypes.byref(cnt)), "msc_debug_set")
        return out
