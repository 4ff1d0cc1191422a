"""Seeded synthetic workloads: arms, obstacle scenes, start poses, targets.

This module only draws random numbers and assembles them into inputs.  It holds
none of the solver's arithmetic (no kinematics, rounding, rasterisation or
search).  Where a workload needs a valid pose or the end point of a pose, the
caller passes a ``pose_fn`` that answers ``(valid, end_voxel)`` for a batch of
poses, so the GPU library and the CPU oracle each build the same inputs from the
same draws with their own arithmetic.

The paper publishes no scene geometry (its figures show "blocks" with dilated
boundaries, Figs 1 and 4), so every scene here is synthetic: axis-aligned boxes
with integer corners and spheres with integer centres and radii, placed
uniformly in the grid.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

YAW, PITCH = 0, 1


@dataclass
class Arm:
    """A serial chain.  Angles are integer centidegrees; ``step_cdeg`` divides 36000."""

    types: List[int]
    lens: List[int]
    lo_cdeg: List[int]
    hi_cdeg: List[int]
    step_cdeg: int
    base: Tuple[int, int, int]
    samples: int = 8
    az0_cdeg: int = 0
    el0_cdeg: int = 9000

    @property
    def dof(self) -> int:
        return len(self.types)

    @property
    def na(self) -> int:
        return 36000 // self.step_cdeg

    def lo_steps(self) -> np.ndarray:
        return np.array(self.lo_cdeg, np.int64) // self.step_cdeg

    def hi_steps(self) -> np.ndarray:
        return np.array(self.hi_cdeg, np.int64) // self.step_cdeg


@dataclass
class Scene:
    n: int                      # grid edge (voxels 0..n-1 per axis)
    dilate: int                 # dilation radius in voxels
    boxes: np.ndarray           # (k, 6) int32: lo x,y,z then extent x,y,z
    spheres: np.ndarray         # (k, 4) int32: centre x,y,z then radius


@dataclass
class Query:
    arm: Arm
    scene: Scene
    target: Tuple[int, int, int]
    start: Optional[np.ndarray] = None   # joint values in steps (path queries)
    waypoints: int = 0                   # number of moves W (path queries)
    max_delta: int = 0                   # max joint change per move, in steps
    seed: Tuple[int, ...] = field(default_factory=tuple)


def rng_for(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(key)))


# --------------------------------------------------------------------------
# Arms of the workloads
# --------------------------------------------------------------------------

def arm_c1() -> Arm:
    """3-DOF arm: base yaw 0..350 deg, then two pitch joints -90..90 deg, 10 deg steps,
    segments 10/8/6 voxels, base (32,32,0) in a 64^3 grid."""
    return Arm(types=[YAW, PITCH, PITCH], lens=[10, 8, 6],
               lo_cdeg=[0, -9000, -9000], hi_cdeg=[35000, 9000, 9000],
               step_cdeg=1000, base=(32, 32, 0))


C2_LENS = [30, 30, 25, 25, 20, 20, 15, 10]


def arm_chain(dof: int, lens: Sequence[int], step_cdeg: int, limit_cdeg: int,
              base: Tuple[int, int, int]) -> Arm:
    """Alternating yaw / pitch chain starting with yaw, symmetric joint limits."""
    types = [YAW if k % 2 == 0 else PITCH for k in range(dof)]
    return Arm(types=types, lens=list(lens[:dof]),
               lo_cdeg=[-limit_cdeg] * dof, hi_cdeg=[limit_cdeg] * dof,
               step_cdeg=step_cdeg, base=base)


def arm_c2() -> Arm:
    """8-DOF alternating yaw/pitch chain, segments 30,30,25,25,20,20,15,10 voxels,
    joint limits +-170 deg in 5 deg steps, base at the floor centre of a 256^3 grid."""
    return arm_chain(8, C2_LENS, 500, 17000, (128, 128, 0))


# The paper's own arm model gives every segment two degrees of freedom at its proximal
# end (azimuth and elevation, "Joint Angular Velocities"); eight DOF = four segments
# ("The selection process for an 8DOF arm").  Here a segment is a zero-length yaw link
# followed by the pitch joint that carries it.  Lengths: the 8-DOF chain's, summed in
# pairs.
GMS_LENS = [60, 50, 40, 25]


def arm_gms(lens: Sequence[int] = GMS_LENS, step_cdeg: int = 500, limit_cdeg: int = 17000,
            base: Tuple[int, int, int] = (128, 128, 0)) -> Arm:
    """Two joints per segment: (yaw, length 0) then (pitch, length L), symmetric limits."""
    types, L = [], []
    for l in lens:
        types += [YAW, PITCH]
        L += [0, int(l)]
    k = len(types)
    return Arm(types=types, lens=L, lo_cdeg=[-limit_cdeg] * k, hi_cdeg=[limit_cdeg] * k,
               step_cdeg=step_cdeg, base=base)


def arm_virtual(lens: Sequence[int], step_cdeg: int = 500, limit_cdeg: int = 17000,
                base: Tuple[int, int, int] = (0, 0, 0)) -> Arm:
    """A virtual arm for paths between arbitrary poses ("Path between Arbitrary Poses"):
    a few segments that can each point anywhere (two joints per segment, as arm_gms),
    rooted where the path starts (the base is replaced by the caller).  The limits are
    the largest multiple of the step within limit_cdeg."""
    return arm_gms(lens, step_cdeg, (limit_cdeg // step_cdeg) * step_cdeg, base)


def scaled_lens(n: int, dof: int) -> List[int]:
    """Prefix of the 8-DOF chain with lengths scaled by n/256, halves rounded up."""
    return [int(np.floor(l * n / 256 + 0.5)) for l in C2_LENS[:dof]]


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------

def _clear_of_column(lo, hi, pad, base, height) -> bool:
    """True if the box [lo-pad, hi+pad] (inclusive, per axis) misses the vertical
    column of voxels base + (0, 0, 0..height).  A plain interval test that keeps the
    first segment's column (it always points up) free of obstacles."""
    if base[0] < lo[0] - pad or base[0] > hi[0] + pad:
        return True
    if base[1] < lo[1] - pad or base[1] > hi[1] + pad:
        return True
    if base[2] + height < lo[2] - pad or base[2] > hi[2] + pad:
        return True
    return False


def random_scene(rng: np.random.Generator, n: int, dilate: int, nbox: int, box_edge: Tuple[int, int],
                 nsph: int = 0, sph_r: Tuple[int, int] = (1, 1),
                 base: Tuple[int, int, int] = (0, 0, 0), column: int = 0,
                 max_tries: int = 10000) -> Scene:
    """Boxes with independent integer edges uniform in box_edge (inclusive) and a lo
    corner uniform such that the box lies in the grid; spheres with integer centre
    uniform in the grid and integer radius uniform in sph_r.  An obstacle whose
    dilated bounding box touches the base column (height ``column``) is redrawn."""
    boxes = []
    tries = 0
    while len(boxes) < nbox:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place boxes clear of the base")
        ext = rng.integers(box_edge[0], box_edge[1] + 1, size=3)
        ext = np.minimum(ext, n)
        lo = np.array([rng.integers(0, n - e + 1) for e in ext])
        hi = lo + ext - 1
        if not _clear_of_column(lo, hi, dilate, base, column):
            continue
        boxes.append(np.concatenate([lo, ext]))
    spheres = []
    tries = 0
    while len(spheres) < nsph:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place spheres clear of the base")
        c = rng.integers(0, n, size=3)
        r = int(rng.integers(sph_r[0], sph_r[1] + 1))
        if not _clear_of_column(c, c, r + dilate, base, column):
            continue
        spheres.append(np.array([c[0], c[1], c[2], r]))
    return Scene(n=n, dilate=dilate,
                 boxes=np.array(boxes, np.int32).reshape(-1, 6),
                 spheres=np.array(spheres, np.int32).reshape(-1, 4))


def scene_c1(seed: int = 0) -> Scene:
    """64^3 grid, 4 boxes with edges uniform 3..10, no dilation."""
    arm = arm_c1()
    return random_scene(rng_for(1, seed, 0), 64, 0, 4, (3, 10), base=arm.base, column=arm.lens[0])


def scene_c2(seed: int = 0) -> Scene:
    """256^3 grid, 32 boxes (edges 5..40) + 8 spheres (radius 4..20), dilation 2."""
    arm = arm_c2()
    return random_scene(rng_for(2, seed, 0), 256, 2, 32, (5, 40), 8, (4, 20),
                        base=arm.base, column=arm.lens[0])


def scene_gms(seed: int = 0) -> Scene:
    """The 256^3 scenes of the 8-DOF chain (boxes, spheres, dilation 2), with the column
    above the base kept clear to the first segment's length."""
    arm = arm_gms()
    return random_scene(rng_for(6, seed, 0), 256, 2, 32, (5, 40), 8, (4, 20),
                        base=arm.base, column=max(arm.lens))


# --------------------------------------------------------------------------
# Poses and targets
# --------------------------------------------------------------------------

PoseFn = Callable[[np.ndarray], Tuple[np.ndarray, np.ndarray]]
"""pose_fn(q[count, dof]) -> (valid[count] bool, end[count, 3] int)."""


def candidate_poses(rng: np.random.Generator, arm: Arm, count: int,
                    lo: Optional[np.ndarray] = None, hi: Optional[np.ndarray] = None) -> np.ndarray:
    lo = arm.lo_steps() if lo is None else lo
    hi = arm.hi_steps() if hi is None else hi
    cols = [rng.integers(lo[k], hi[k] + 1, size=count) for k in range(arm.dof)]
    return np.stack(cols, axis=1).astype(np.int32)


def first_valid_pose(rng: np.random.Generator, arm: Arm, pose_fn: PoseFn,
                     batch: int = 4096, max_batches: int = 64) -> Tuple[np.ndarray, np.ndarray, int]:
    """Uniform joint values, redrawn until the caller's pose_fn calls one valid.
    Returns (pose, end voxel, index of the accepted candidate)."""
    for b in range(max_batches):
        q = candidate_poses(rng, arm, batch)
        valid, end = pose_fn(q)
        hits = np.flatnonzero(valid)
        if hits.size:
            i = int(hits[0])
            return q[i].copy(), np.asarray(end[i]).copy(), b * batch + i
    raise RuntimeError("no valid pose found")


def walk_target(rng: np.random.Generator, arm: Arm, start: np.ndarray, waypoints: int, delta: int,
                pose_fn: PoseFn, redraws: int = 8) -> Tuple[np.ndarray, np.ndarray]:
    """A waypoints-move walk from start: each joint steps towards a uniform goal pose
    inside the reachable window with probability 3/4, else by a uniform value in
    {-delta, 0, +delta}; a move whose pose pose_fn rejects is redrawn (up to
    ``redraws`` times, then the arm stays).  Returns (end pose, its end voxel): a
    target that a path of ``waypoints`` moves can reach by construction."""
    lo, hi = arm.lo_steps(), arm.hi_steps()
    span = waypoints * delta
    wlo = np.maximum(lo, start - span)
    whi = np.minimum(hi, start + span)
    goal = np.array([rng.integers(wlo[k], whi[k] + 1) for k in range(arm.dof)], np.int64)
    q = np.asarray(start, np.int64).copy()
    for _ in range(waypoints):
        moved = False
        for _r in range(redraws):
            toward = rng.random(arm.dof) < 0.75
            rand_step = rng.integers(-1, 2, size=arm.dof) * delta
            step = np.where(toward, np.clip(goal - q, -delta, delta), rand_step)
            cand = np.clip(q + step, lo, hi)
            valid, _ = pose_fn(cand[None, :].astype(np.int32))
            if bool(valid[0]):
                q = cand
                moved = True
                break
        if not moved:
            pass  # stay: the current pose is valid
    valid, end = pose_fn(q[None, :].astype(np.int32))
    assert bool(valid[0])
    return q.astype(np.int32), np.asarray(end[0]).astype(np.int64)


def query_c1(seed: int, pose_fn_for: Callable[[Arm, Scene], PoseFn]) -> Query:
    """Single reach query: target = end voxel of a uniformly drawn valid pose."""
    arm, scene = arm_c1(), scene_c1(seed)
    pf = pose_fn_for(arm, scene)
    _, end, _ = first_valid_pose(rng_for(1, seed, 1), arm, pf)
    return Query(arm=arm, scene=scene, target=tuple(int(v) for v in end), seed=(1, seed))


def query_c2(seed: int, pose_fn_for: Callable[[Arm, Scene], PoseFn], waypoints: int = 16,
             delta: int = 1) -> Query:
    """Reach + path query: random valid start pose, 16 moves of at most one step
    (5 deg) per joint, target at the end of a feasible walk from the start."""
    arm, scene = arm_c2(), scene_c2(seed)
    pf = pose_fn_for(arm, scene)
    start, _, _ = first_valid_pose(rng_for(2, seed, 1), arm, pf)
    _, end = walk_target(rng_for(2, seed, 2), arm, start, waypoints, delta, pf)
    return Query(arm=arm, scene=scene, target=tuple(int(v) for v in end), start=start,
                 waypoints=waypoints, max_delta=delta, seed=(2, seed))


def query_gms(seed: int, pose_fn_for: Callable[[Arm, Scene], PoseFn], waypoints: int = 16,
              delta: int = 1) -> Query:
    """Reach + path query of the two-DOF-per-segment arm, drawn like the 8-DOF chain's:
    random valid start, target at the end of a feasible 16-move walk."""
    arm, scene = arm_gms(), scene_gms(seed)
    pf = pose_fn_for(arm, scene)
    start, _, _ = first_valid_pose(rng_for(6, seed, 1), arm, pf)
    _, end = walk_target(rng_for(6, seed, 2), arm, start, waypoints, delta, pf)
    return Query(arm=arm, scene=scene, target=tuple(int(v) for v in end), start=start,
                 waypoints=waypoints, max_delta=delta, seed=(6, seed))


# --------------------------------------------------------------------------
# Batched and larger workloads
# --------------------------------------------------------------------------

def scene_c3(scene_seed: int, n: Optional[int] = None) -> Scene:
    """One of the 64 scenes of the batched-reach workload: grid 128^3 or 256^3 (uniform),
    10..60 boxes with edges 5..40 scaled by n/256, dilation round(2 n/256)."""
    rng = rng_for(3, scene_seed, 0)
    if n is None:
        n = int(rng.choice([128, 256]))
    else:
        rng.choice([128, 256])
    nbox = int(rng.integers(10, 61))
    lo_e = max(1, int(round(5 * n / 256)))
    hi_e = max(lo_e, int(round(40 * n / 256)))
    dilate = int(round(2 * n / 256))
    base = (n // 2, n // 2, 0)
    return random_scene(rng, n, dilate, nbox, (lo_e, hi_e), base=base, column=scaled_lens(n, 1)[0])


def queries_c3(pose_fn_for: Callable[[Arm, Scene], PoseFn], scenes: int = 64, per_scene: int = 8,
               n: Optional[int] = None, max_dof: int = 8, step_cdeg: int = 500) -> List[Query]:
    """Batched reach poses: per scene, `per_scene` queries with DOF uniform 5..max_dof
    (prefix of the 8-DOF chain, lengths scaled by n/256), joints +-170 deg; the target is
    the end voxel (inside the grid) of a uniformly drawn pose, valid or not, so some
    queries have no answer."""
    out = []
    for s in range(scenes):
        sc = scene_c3(s, n)
        rng = rng_for(3, s, 1)
        for j in range(per_scene):
            dof = int(rng.integers(5, max_dof + 1))
            arm = arm_chain(dof, scaled_lens(sc.n, dof), step_cdeg, 17000, (sc.n // 2, sc.n // 2, 0))
            pf = pose_fn_for(arm, sc)
            while True:  # redraw poses whose end voxel lies outside the grid
                q = candidate_poses(rng, arm, 1)
                _, end = pf(q)
                end = np.asarray(end)[0]
                if np.all(end >= 0) and np.all(end < sc.n):
                    break
            out.append(Query(arm=arm, scene=sc, target=tuple(int(v) for v in end), seed=(3, s, j)))
    return out


def queries_c4(pose_fn_for: Callable[[Arm, Scene], PoseFn], scenes: int = 8, per_scene: int = 32,
               n: int = 512, step_cdeg: int = 250, lens_scale: float = 2.0, w_range: Tuple[int, int] = (8, 64),
               dof: int = 8) -> List[Query]:
    """Batched paths: 8 shared 512^3 scenes (40 boxes with edges 10..80, 16 spheres of
    radius 8..40, dilation 4), 8-DOF chain with the segment lengths doubled, 2.5 deg
    steps, +-170 deg, 8..64 waypoints of at most one step per joint.  The scale knobs
    give the shrunken variants used by the parity tests."""
    out = []
    f = n / 512
    for s in range(scenes):
        rng = rng_for(4, s, 0)
        lens = [max(1, int(round(l * lens_scale * f))) for l in C2_LENS[:dof]]
        base = (n // 2, n // 2, 0)
        sc = random_scene(rng, n, max(0, int(round(4 * f))), 40, (max(1, int(10 * f)), max(1, int(80 * f))),
                          16, (max(1, int(8 * f)), max(1, int(40 * f))), base=base, column=lens[0])
        arm = arm_chain(dof, lens, step_cdeg, 17000, base)
        pf = pose_fn_for(arm, sc)
        for j in range(per_scene):
            r = rng_for(4, s, 1 + j)
            start, _, _ = first_valid_pose(r, arm, pf, batch=1024)
            W = int(r.integers(w_range[0], w_range[1] + 1))
            _, end = walk_target(r, arm, start, W, 1, pf)
            out.append(Query(arm=arm, scene=sc, target=tuple(int(v) for v in end), start=start, waypoints=W,
                             max_delta=1, seed=(4, s, j)))
    return out
