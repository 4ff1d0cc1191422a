"""Serving loop with dynamic obstacles and midcourse replanning ("Dynamic Obstacles").

A real-time loop of logical ticks (10 ms each).  The library does the work of a tick;
this module only draws the workload and drives the clock:

* every tick, each scene's moving boxes advance (constant velocity in 1/1024-voxel
  fixed point, reflected at the walls) and ``msc_scene_set_dynamic`` writes the
  scene's grid of that tick (static + moving obstacles) into one of the scene's
  resident grids of recent ticks, asynchronously;
* ``msc_server_step`` then re-validates, on the library's side, the remaining
  waypoints of every path executing on the server's logical clock (one waypoint every
  ``ticks_per_waypoint`` ticks: the paper's arm traverses a waypoint in about 83 ms)
  and queues a replan of the rest of a path from its current pose when a waypoint
  ahead collides;
* requests arrive as a Poisson process (70% reach pose, 30% reach + path) and are
  submitted to the library's server (continuous batching over worker lanes); each is
  bound to the grid of its submission tick, so its result does not depend on what else
  is in flight.  Start poses and targets are drawn before the loop against the static
  obstacles; at their tick a moving box may block the start (E_ARG) or the target
  (NO_REACH), which are served outcomes like any other.  Solved paths execute on the
  server;
* latency of every request (submission to completion, measured by the library) is
  recorded per class: reach, path, and the replans the server issued; with
  ``max_pending`` the server refuses new requests while that many wait for a lane
  (admission by queue depth), and the refused ones are counted as shed.

Random draws come from `synth`; kinematics, rasterisation, re-validation and search
all run in the library.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

from . import msc, synth

FIX = 1024  # fixed-point scale of moving-box positions


@dataclass
class Movers:
    """The moving boxes of one scene: lo corners in fixed point, velocities per tick,
    integer extents."""
    pos: np.ndarray     # (k, 3) int64, x FIX
    vel: np.ndarray     # (k, 3) int64, x FIX per tick
    ext: np.ndarray     # (k, 3) int64

    def step(self, n: int):
        hi_lim = (n - self.ext) * FIX
        p = self.pos + self.vel
        lo_hit = p < 0
        hi_hit = p > hi_lim
        p = np.where(lo_hit, -p, p)
        p = np.where(hi_hit, 2 * hi_lim - p, p)
        self.vel = np.where(lo_hit | hi_hit, -self.vel, self.vel)
        self.pos = p

    def boxes(self) -> np.ndarray:
        """(k, 6) int32: lo corner then extent, as msc_box."""
        return np.ascontiguousarray(np.concatenate([self.pos // FIX, self.ext], axis=1).astype(np.int32))


@dataclass
class DynScene:
    static: synth.Scene
    movers: Movers

    def at(self, boxes: np.ndarray) -> synth.Scene:
        """The scene with the given moving boxes added to the static ones."""
        return synth.Scene(n=self.static.n, dilate=self.static.dilate,
                           boxes=np.concatenate([self.static.boxes, boxes]) if len(boxes) else self.static.boxes,
                           spheres=self.static.spheres)


def make_dyn_scene(seed: int, n: int = 256, column: int = 30) -> DynScene:
    """C2-style static obstacles plus 1..8 moving boxes (edges 10..30 voxels, speed
    0.5..3 voxels per tick in a uniform direction), sizes scaled by n / 256."""
    f = n / 256
    base = (n // 2, n // 2, 0)
    static = synth.random_scene(synth.rng_for(5, seed, 0), n, int(round(2 * f)), 32,
                                (max(1, int(round(5 * f))), max(1, int(round(40 * f)))), 8,
                                (max(1, int(round(4 * f))), max(1, int(round(20 * f)))), base=base, column=column)
    rng = synth.rng_for(5, seed, 1)
    k = int(rng.integers(1, 9))
    pos, vel, ext = [], [], []
    for _ in range(k):
        e = np.minimum(rng.integers(max(1, int(round(10 * f))), max(1, int(round(30 * f))) + 1, size=3), n)
        lo = np.array([rng.integers(0, n - v + 1) for v in e], np.int64) * FIX
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        speed = rng.uniform(0.5, 3.0) * f
        pos.append(lo)
        vel.append(np.round(d * speed * FIX).astype(np.int64))
        ext.append(e.astype(np.int64))
    return DynScene(static=static, movers=Movers(np.array(pos), np.array(vel), np.array(ext)))


@dataclass
class Template:
    kind: str                  # reach / path
    scene_idx: int
    arm: synth.Arm
    target: Tuple[int, int, int]
    start: Optional[np.ndarray] = None
    waypoints: int = 0


def c5_arm(dof: int, n: int = 256) -> synth.Arm:
    """The serving workload's arms: DOF-long prefixes of the 8-DOF chain, 5 deg steps."""
    lens = synth.C2_LENS if n == 256 else synth.scaled_lens(n, 8)
    return synth.arm_chain(dof, lens, 500, 17000, (n // 2, n // 2, 0))


def draw_templates(solver: msc.Solver, dyn: List[DynScene], count: int, seed: int, path_frac: float = 0.3,
                   dof_range: Tuple[int, int] = (6, 8), w_range: Tuple[int, int] = (8, 32),
                   arm_for: Optional[Callable[[int], synth.Arm]] = None):
    """Request templates against the static obstacles: arms of DOF in dof_range; reach
    targets are ends of valid poses; path targets ends of feasible walks of w_range
    moves of one step."""
    rng = synth.rng_for(7, seed)
    n = dyn[0].static.n
    arm_for = arm_for or (lambda d: c5_arm(d, n))
    statics = [solver.scene(d.static) for d in dyn]
    out = []
    for _ in range(count):
        si = int(rng.integers(0, len(dyn)))
        dof = int(rng.integers(dof_range[0], dof_range[1] + 1))
        arm = arm_for(dof)
        pf = lambda q, sc=statics[si], a=arm: solver.pose_check(sc, a, q)  # noqa: E731
        if rng.random() < path_frac:
            start, _, _ = synth.first_valid_pose(rng, arm, pf, batch=512)
            W = int(rng.integers(w_range[0], w_range[1] + 1))
            _, target = synth.walk_target(rng, arm, start, W, 1, pf, redraws=2)
            out.append(Template("path", si, arm, tuple(int(v) for v in target), start, W))
        else:
            _, end, _ = synth.first_valid_pose(rng, arm, pf, batch=512)
            out.append(Template("reach", si, arm, tuple(int(v) for v in end)))
    return out


@dataclass
class Request:
    kind: str                  # reach / path
    spec: msc.QuerySpec
    ticket: int = 0
    scene_idx: int = 0


@dataclass
class ServeReport:
    latencies: Dict[str, List[float]] = field(default_factory=lambda: {"reach": [], "path": [], "replan": []})
    statuses: Dict[str, Dict[int, int]] = field(default_factory=dict)
    served: int = 0
    submitted: int = 0
    wall_s: float = 0.0
    ticks: int = 0
    late_ticks: int = 0        # ticks started more than one tick late (the loop fell behind)
    stale_ticks: int = 0       # ticks whose grid could not be written (every grid of a tick in use)
    replans: int = 0
    stopped: int = 0
    shed: int = 0              # requests the server refused for its queue depth
    unserved: int = 0          # requests or replans still in flight when the drain timed out
    tick_ms: List[float] = field(default_factory=list)   # host time spent in each tick's work
    done_log: List[tuple] = field(default_factory=list)   # (kind, scene_idx, tick, status, result, spec)
    replan_log: List[dict] = field(default_factory=list)

    def count(self, kind: str, st: int):
        self.statuses.setdefault(kind, {})
        self.statuses[kind][st] = self.statuses[kind].get(st, 0) + 1

    def summary(self) -> dict:
        out = {"served": self.served, "submitted": self.submitted, "wall_s": round(self.wall_s, 3),
               "solves_per_s": round(self.served / max(self.wall_s, 1e-9), 2), "ticks": self.ticks,
               "late_ticks": self.late_ticks, "stale_ticks": self.stale_ticks, "replans": self.replans,
               "stopped": self.stopped, "shed": self.shed}
        if self.tick_ms:
            t = np.array(self.tick_ms)
            out["tick_work_ms"] = {"p50": round(float(np.percentile(t, 50)), 3),
                                   "p99": round(float(np.percentile(t, 99)), 3)}
        for k, v in self.latencies.items():
            if v:
                a = np.array(v)
                out[k] = {"n": len(v), "p50_ms": round(float(np.percentile(a, 50)), 3),
                          "p99_ms": round(float(np.percentile(a, 99)), 3)}
        out["statuses"] = self.statuses
        return out


class ServingLoop:
    def __init__(self, solver: msc.Solver, nscenes: int = 16, seed: int = 0, rate: float = 500.0,
                 tick_ms: float = 10.0, path_frac: float = 0.3, ticks_per_waypoint: int = 8,
                 keep_log: bool = False, templates: int = 2000, n: int = 256,
                 dof_range: Tuple[int, int] = (6, 8), w_range: Tuple[int, int] = (8, 32),
                 arm_for: Optional[Callable[[int], synth.Arm]] = None, tick_grids: int = 24,
                 max_pending: int = 0):
        self.solver = solver
        self.rng = synth.rng_for(6, seed)
        column = (arm_for(dof_range[1]) if arm_for else c5_arm(dof_range[1], n)).lens[0]
        self.dyn = [make_dyn_scene(seed * 1000 + i, n, column) for i in range(nscenes)]
        self.templates = draw_templates(solver, self.dyn, templates, seed, path_frac, dof_range, w_range, arm_for)
        self.scenes = [solver.scene(d.static, ticks=tick_grids) for d in self.dyn]
        self.next_template = 0
        self.rate = rate
        self.tick_ms = tick_ms
        self.tpw = ticks_per_waypoint
        self.keep_log = keep_log
        self.tick = 0
        self.pending: List[Request] = []
        self.report = ServeReport()
        self.mover_log: Dict[int, List[np.ndarray]] = {}   # tick -> moving boxes per scene (keep_log)
        self.replans_inflight = 0
        self.max_pending = max_pending   # > 0: the server sheds submissions beyond this queue depth

    # -- scenes -----------------------------------------------------------------
    def advance_tick(self):
        """Move the boxes, write every scene's grid of this tick, then let the server
        re-validate the executing paths on them."""
        if self.tick > 0:
            for d in self.dyn:
                d.movers.step(d.static.n)
        boxes = [d.movers.boxes() for d in self.dyn]
        if self.keep_log:
            self.mover_log[self.tick] = boxes
        lib = self.solver.lib
        for sc, b in zip(self.scenes, boxes):
            rc = lib.msc_scene_set_dynamic(sc.handle, b.ctypes.data_as(ctypes.POINTER(msc.MscBox)), len(b),
                                           self.tick)
            if rc == msc.E_CAPACITY:
                self.report.stale_ticks += 1   # queries keep solving on the previous grid
            else:
                self.solver._check(rc, "msc_scene_set_dynamic")
        rep = self.solver.server_step(self.tick)
        self.report.replans += rep["replans"]
        self.report.stopped += rep["stopped"]
        self.replans_inflight += rep["replans"]

    def scene_at(self, scene_idx: int, tick: int) -> synth.Scene:
        """The obstacles of a scene at a logical tick (needs keep_log)."""
        return self.dyn[scene_idx].at(self.mover_log[tick][scene_idx])

    # -- requests ---------------------------------------------------------------
    def draw_request(self) -> Request:
        tp = self.templates[self.next_template % len(self.templates)]
        self.next_template += 1
        scene = self.scenes[tp.scene_idx]
        if tp.kind == "path":
            spec = msc.QuerySpec(scene, tp.arm, tp.target, start=tp.start, waypoints=tp.waypoints, delta=1,
                                 execute_ticks=self.tpw)
            return Request("path", spec, scene_idx=tp.scene_idx)
        return Request("reach", msc.QuerySpec(scene, tp.arm, tp.target), scene_idx=tp.scene_idx)

    def submit(self, req: Request):
        req.ticket = self.solver.submit(req.spec, shed=self.max_pending > 0)
        if req.ticket is None:
            self.report.shed += 1
            return
        self.pending.append(req)
        self.report.submitted += 1

    def collect(self):
        still = []
        for req in self.pending:
            if not self.solver.poll(req.ticket):
                still.append(req)
                continue
            st, res, lat = req.spec.result()
            self.report.latencies[req.kind].append(lat)
            self.report.count(req.kind, st)
            self.report.served += 1
            if self.keep_log:
                self.report.done_log.append((req.kind, req.scene_idx, req.spec.tick, st, res, req.spec))
        self.pending = still
        for r in self.solver.take_replans():
            self.replans_inflight -= 1
            self.report.latencies["replan"].append(r["latency_ms"])
            self.report.count("replan", r["status"])
            self.report.served += 1
            if self.keep_log:
                r["scene_idx"] = next(i for i, sc in enumerate(self.scenes) if sc.handle.value == r["scene"])
                self.report.replan_log.append(r)

    # -- loop -------------------------------------------------------------------
    def run(self, seconds: float, warmup_s: float = 1.0, drain_s: float = 30.0) -> ServeReport:
        self.solver.server_start()
        if self.max_pending:
            self.solver.server_set_limit(self.max_pending)
        try:
            t_begin = time.perf_counter()
            next_tick_at = t_begin
            measuring_from = t_begin + warmup_s
            t_end = measuring_from + seconds
            measuring = False
            while True:
                now = time.perf_counter()
                if not measuring and now >= measuring_from:
                    measuring = True
                    self.report = ServeReport(done_log=self.report.done_log if self.keep_log else [],
                                              replan_log=self.report.replan_log if self.keep_log else [])
                    measure_t0 = now
                if now >= t_end:
                    break
                if now >= next_tick_at:
                    if now - next_tick_at > self.tick_ms / 1e3:
                        self.report.late_ticks += 1
                    self.advance_tick()
                    arrivals = int(self.rng.poisson(self.rate * self.tick_ms / 1e3))
                    for _ in range(arrivals):
                        self.submit(self.draw_request())
                    self.tick += 1
                    self.report.ticks += 1
                    self.report.tick_ms.append((time.perf_counter() - now) * 1e3)
                    next_tick_at += self.tick_ms / 1e3
                self.collect()
                time.sleep(0.0002)
            # drain what is in flight (the clock stops with the measured window, so no
            # further replans are issued)
            t_drain = time.perf_counter()
            while (self.pending or self.replans_inflight > 0) and time.perf_counter() - t_drain < drain_s:
                self.collect()
                time.sleep(0.0005)
            self.report.wall_s = time.perf_counter() - measure_t0
            self.report.unserved = len(self.pending) + self.replans_inflight
        finally:
            self.solver.server_stop()
        return self.report
