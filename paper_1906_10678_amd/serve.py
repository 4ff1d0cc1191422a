"""Serving loop with dynamic obstacles and midcourse replanning ("Dynamic Obstacles").

A real-time loop of logical ticks (10 ms each):

* every tick, each scene's moving boxes advance (constant velocity in 1/1024-voxel
  fixed point, reflected at the walls) and the scene is rasterised again into a new
  device grid (static + moving obstacles): the grid of that tick;
* requests arrive as a Poisson process (70% reach pose, 30% reach + path) and are
  submitted to the library's server (continuous batching over worker lanes), each
  against the grid of its arrival tick, so its result does not depend on what else is
  in flight.  Their start poses and targets are drawn before the loop against the
  static obstacles; at their tick a moving box may block the start (E_ARG) or the
  target (NO_REACH), which are served outcomes like any other;
* a finished path starts to execute: the arm advances one waypoint every
  `ticks_per_waypoint` ticks ("each waypoint ... traversed in approximately 83 msec");
  at every tick its remaining waypoints are re-validated on the GPU against the
  current grid, and if one collides the remaining part is replanned from the current
  pose to the same target (the paper's midcourse replanning);
* latency of every request (submission to completion, wall clock) is recorded per
  class: reach, path, replan.

Random draws come from `synth`; kinematics, rasterisation and search all run in the
library.  A request that finds no answer (NO_REACH / NO_PATH: the target is blocked
at that tick) still counts as served.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import msc, synth

FIX = 1024  # fixed-point scale of moving-box positions


@dataclass
class MovingBox:
    pos: np.ndarray     # lo corner, fixed point (int64, x FIX)
    vel: np.ndarray     # fixed point per tick
    ext: np.ndarray     # integer extent

    def step(self, n: int):
        hi_lim = (n - self.ext) * FIX
        self.pos = self.pos + self.vel
        for a in range(3):
            if self.pos[a] < 0:
                self.pos[a] = -self.pos[a]
                self.vel[a] = -self.vel[a]
            elif self.pos[a] > hi_lim[a]:
                self.pos[a] = 2 * hi_lim[a] - self.pos[a]
                self.vel[a] = -self.vel[a]

    def box(self) -> np.ndarray:
        return np.concatenate([self.pos // FIX, self.ext]).astype(np.int32)


@dataclass
class DynScene:
    static: synth.Scene
    movers: List[MovingBox]

    def at_tick(self) -> synth.Scene:
        boxes = np.concatenate([self.static.boxes] + [m.box()[None, :] for m in self.movers]) \
            if self.movers else self.static.boxes
        return synth.Scene(n=self.static.n, dilate=self.static.dilate, boxes=boxes, spheres=self.static.spheres)


def make_dyn_scene(seed: int, n: int = 256) -> DynScene:
    """C2-style static obstacles plus 1..8 moving boxes (edges 10..30 voxels, speed
    0.5..3 voxels per tick in a uniform direction)."""
    arm = synth.arm_c2()
    static = synth.random_scene(synth.rng_for(5, seed, 0), n, 2, 32, (5, 40), 8, (4, 20), base=arm.base,
                                column=arm.lens[0])
    rng = synth.rng_for(5, seed, 1)
    movers = []
    for _ in range(int(rng.integers(1, 9))):
        ext = rng.integers(10, 31, size=3)
        lo = np.array([rng.integers(0, n - e + 1) for e in ext], np.int64) * FIX
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        speed = rng.uniform(0.5, 3.0)
        vel = np.round(d * speed * FIX).astype(np.int64)
        movers.append(MovingBox(pos=lo, vel=vel, ext=ext.astype(np.int64)))
    return DynScene(static=static, movers=movers)


@dataclass
class Executing:
    path: np.ndarray           # (W+1, dof) steps
    target: Tuple[int, int, int]
    arm: synth.Arm
    scene_idx: int
    start_tick: int
    replans: int = 0


@dataclass
class Template:
    kind: str                  # reach / path
    scene_idx: int
    arm: synth.Arm
    target: Tuple[int, int, int]
    start: Optional[np.ndarray] = None
    waypoints: int = 0


def draw_templates(solver: msc.Solver, dyn: List["DynScene"], count: int, seed: int, path_frac: float = 0.3):
    """Request templates against the static obstacles: DOF 6..8 prefixes of the 8-DOF
    chain; reach targets are ends of valid poses; path targets ends of feasible walks of
    8..32 moves of one step (5 deg)."""
    rng = synth.rng_for(7, seed)
    statics = [solver.scene(d.static) for d in dyn]
    base = synth.arm_c2().base
    out = []
    for _ in range(count):
        si = int(rng.integers(0, len(dyn)))
        dof = int(rng.integers(6, 9))
        arm = synth.arm_chain(dof, synth.C2_LENS, 500, 17000, base)
        pf = lambda q, sc=statics[si], a=arm: solver.pose_check(sc, a, q)  # noqa: E731
        if rng.random() < path_frac:
            start, _, _ = synth.first_valid_pose(rng, arm, pf, batch=512)
            W = int(rng.integers(8, 33))
            _, target = synth.walk_target(rng, arm, start, W, 1, pf, redraws=2)
            out.append(Template("path", si, arm, tuple(int(v) for v in target), start, W))
        else:
            _, end, _ = synth.first_valid_pose(rng, arm, pf, batch=512)
            out.append(Template("reach", si, arm, tuple(int(v) for v in end)))
    return out


@dataclass
class Request:
    kind: str                  # reach / path / replan
    tick: int
    spec: msc.QuerySpec
    ticket: int = 0
    submitted: float = 0.0
    execute: Optional[Executing] = None


@dataclass
class ServeReport:
    latencies: Dict[str, List[float]] = field(default_factory=lambda: {"reach": [], "path": [], "replan": []})
    statuses: Dict[str, Dict[int, int]] = field(default_factory=dict)
    served: int = 0
    submitted: int = 0
    wall_s: float = 0.0
    ticks: int = 0
    replans: int = 0
    done_log: List[tuple] = field(default_factory=list)   # (kind, tick, status, result, spec)

    def summary(self) -> dict:
        out = {"served": self.served, "submitted": self.submitted, "wall_s": round(self.wall_s, 3),
               "solves_per_s": round(self.served / max(self.wall_s, 1e-9), 2), "ticks": self.ticks,
               "replans": self.replans}
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
                 keep_log: bool = False, templates: int = 2000):
        self.solver = solver
        self.rng = synth.rng_for(6, seed)
        self.dyn = [make_dyn_scene(seed * 1000 + i) for i in range(nscenes)]
        self.templates = draw_templates(solver, self.dyn, templates, seed, path_frac)
        self.next_template = 0
        self.rate = rate
        self.tick_ms = tick_ms
        self.path_frac = path_frac
        self.tpw = ticks_per_waypoint
        self.keep_log = keep_log
        self.tick = 0
        self.grids: Dict[int, List[msc.Scene]] = {}
        self.pending: List[Request] = []
        self.executing: List[Executing] = []
        self.report = ServeReport()

    # -- scenes -----------------------------------------------------------------
    def advance_tick(self):
        if self.tick > 0:
            for d in self.dyn:
                for m in d.movers:
                    m.step(d.static.n)
        self.grids[self.tick] = [self.solver.scene(d.at_tick()) for d in self.dyn]
        # grids of old ticks are kept alive by the requests that reference them
        for t in [t for t in self.grids if t < self.tick]:
            del self.grids[t]

    # -- requests ---------------------------------------------------------------
    def draw_request(self) -> Request:
        tp = self.templates[self.next_template % len(self.templates)]
        self.next_template += 1
        scene = self.grids[self.tick][tp.scene_idx]
        if tp.kind == "path":
            spec = msc.QuerySpec(scene, tp.arm, tp.target, start=tp.start, waypoints=tp.waypoints, delta=1)
            req = Request("path", self.tick, spec)
            req.execute = Executing(path=None, target=tp.target, arm=tp.arm, scene_idx=tp.scene_idx, start_tick=0)
            return req
        return Request("reach", self.tick, msc.QuerySpec(scene, tp.arm, tp.target))

    def submit(self, req: Request):
        req.submitted = time.perf_counter()
        req.ticket = self.solver.submit(req.spec)
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
            self.report.statuses.setdefault(req.kind, {})
            self.report.statuses[req.kind][st] = self.report.statuses[req.kind].get(st, 0) + 1
            self.report.served += 1
            if self.keep_log:
                self.report.done_log.append((req.kind, req.tick, st, res, req.spec))
            if req.kind in ("path", "replan") and st == msc.OK and req.execute is not None:
                ex = req.execute
                ex.path = res
                ex.start_tick = self.tick
                self.executing.append(ex)
        self.pending = still

    def revalidate(self):
        """Re-check the remaining waypoints of executing paths against this tick's grid
        (one GPU pose check per scene and arm); replan the rest of a path whose remaining
        waypoints collide."""
        live = []
        for ex in self.executing:
            done_wp = (self.tick - ex.start_tick) // self.tpw
            if done_wp < ex.path.shape[0] - 1:
                live.append((ex, done_wp))
        groups: Dict[Tuple[int, int], List[Tuple[Executing, int]]] = {}
        for ex, d in live:
            groups.setdefault((ex.scene_idx, ex.arm.dof), []).append((ex, d))
        verdict = {}
        for (si, dof), items in groups.items():
            rows = np.concatenate([ex.path[d:] for ex, d in items])
            valid, _ = self.solver.pose_check(self.grids[self.tick][si], items[0][0].arm, rows)
            o = 0
            for ex, d in items:
                k = ex.path.shape[0] - d
                verdict[id(ex)] = valid[o:o + k]
                o += k
        keep = []
        for ex, done_wp in live:
            W = ex.path.shape[0] - 1
            valid = verdict[id(ex)]
            scene = self.grids[self.tick][ex.scene_idx]
            if valid.all():
                keep.append(ex)
                continue
            current = ex.path[done_wp]
            if not valid[0]:
                continue  # the arm's current pose is hit: nothing to replan from
            remaining = W - done_wp
            # the new path nearest the rest of the original one ("Dynamic Obstacles")
            spec = msc.QuerySpec(scene, ex.arm, ex.target, start=current, waypoints=remaining, delta=1,
                                 ref=ex.path[done_wp:])
            req = Request("replan", self.tick, spec)
            req.execute = Executing(path=None, target=ex.target, arm=ex.arm, scene_idx=ex.scene_idx,
                                    start_tick=0, replans=ex.replans + 1)
            self.submit(req)
            self.report.replans += 1
        self.executing = keep

    # -- loop -------------------------------------------------------------------
    def run(self, seconds: float, warmup_s: float = 1.0) -> ServeReport:
        self.solver.server_start()
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
                    self.report = ServeReport()
                    measure_t0 = now
                if now >= t_end:
                    break
                if now >= next_tick_at:
                    self.advance_tick()
                    arrivals = int(self.rng.poisson(self.rate * self.tick_ms / 1e3))
                    for _ in range(arrivals):
                        self.submit(self.draw_request())
                    self.revalidate()
                    self.tick += 1
                    self.report.ticks += 1
                    next_tick_at += self.tick_ms / 1e3
                self.collect()
                time.sleep(0.0002)
            # drain
            while self.pending:
                self.collect()
                time.sleep(0.0005)
            self.report.wall_s = time.perf_counter() - measure_t0
        finally:
            self.solver.server_stop()
        return self.report
