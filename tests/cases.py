"""Small seeded cases shared by the oracle pins and the GPU parity tests.

Only random draws live here (through the synth module); the oracle and the GPU
library each compute everything else themselves.
"""
from __future__ import annotations

import numpy as np

from paper_1906_10678_amd import synth


def tiny_arm(rng: np.random.Generator, dof: int, step_cdeg: int = 3000, n: int = 20,
             lens=None, limits=None) -> synth.Arm:
    """Alternating yaw/pitch chain with short segments; base at the floor centre."""
    na = 36000 // step_cdeg
    types = [synth.YAW if k % 2 == 0 else synth.PITCH for k in range(dof)]
    if lens is None:
        lens = [int(v) for v in rng.integers(2, 6, size=dof)]
    lo, hi = [], []
    for k in range(dof):
        if limits is not None:
            l, h = limits[k]
        else:
            span = int(rng.integers(max(1, na // 4), na // 2 + 1))
            l = -span * step_cdeg
            h = int(rng.integers(span // 2, span + 1)) * step_cdeg
        lo.append(l)
        hi.append(h)
    return synth.Arm(types=types, lens=list(lens), lo_cdeg=lo, hi_cdeg=hi, step_cdeg=step_cdeg,
                     base=(n // 2, n // 2, 0))


def tiny_scene(rng: np.random.Generator, n: int, nbox: int, dilate: int = 0, nsph: int = 0,
               base=None, column: int = 0) -> synth.Scene:
    base = base if base is not None else (n // 2, n // 2, 0)
    return synth.random_scene(rng, n, dilate, nbox, (1, max(2, n // 4)), nsph, (1, max(1, n // 8)),
                              base=base, column=column)


def tiny_case(seed: int, dof: int = 3, step_cdeg: int = 3000, n: int = 20, nbox: int = 3,
              dilate: int = 0, nsph: int = 1):
    """(arm, scene, pose draws) for a tiny problem; the target is chosen by the caller
    from the draws with its own pose replay."""
    rng = synth.rng_for(900, seed)
    arm = tiny_arm(rng, dof, step_cdeg, n)
    scene = tiny_scene(rng, n, nbox, dilate, nsph, base=arm.base, column=arm.lens[0])
    return arm, scene, rng


def arm_fields(arm) -> dict:
    return dict(types=list(arm.types), lens=list(arm.lens), lo=list(arm.lo_cdeg), hi=list(arm.hi_cdeg),
                step=arm.step_cdeg, base=tuple(arm.base))


def tiny_gms_arm(rng: np.random.Generator, segments: int, step_cdeg: int = 3000, n: int = 20) -> synth.Arm:
    """The paper's arm model at tiny size: each segment a zero-length yaw link followed by
    a pitch joint carrying the segment (2 DOF per segment), random windows."""
    lens = [int(v) for v in rng.integers(2, 6, size=segments)]
    arm = synth.arm_gms(lens, step_cdeg, 18000, (n // 2, n // 2, 0))
    na = 36000 // step_cdeg
    lo, hi = [], []
    for k in range(arm.dof):
        span = int(rng.integers(max(1, na // 4), na // 2 + 1))
        lo.append(-span * step_cdeg)
        hi.append(int(rng.integers(span // 2, span + 1)) * step_cdeg)
    arm.lo_cdeg, arm.hi_cdeg = lo, hi
    return arm


def tiny_gms_case(seed: int, segments: int = 2, step_cdeg: int = 3000, n: int = 20, nbox: int = 3,
                  dilate: int = 0, nsph: int = 1):
    rng = synth.rng_for(906, seed)
    arm = tiny_gms_arm(rng, segments, step_cdeg, n)
    scene = tiny_scene(rng, n, nbox, dilate, nsph, base=arm.base, column=max(arm.lens))
    return arm, scene, rng
