"""Writes c3_reach.json: the oracle's answers to the full-size batched-reach queries of
scenes 0..15 (128^3 / 256^3 grids, unwindowed joints, 5 deg steps) whose arm has at
most 6 DOF (the oracle needs seconds for those, far longer for 7 and 8 DOF), with a
fingerprint of each query's inputs.

Only the oracle computes these values.  Run from the repository root:
python tests/golden/make_c3_reach.py
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
from make_c2_paths import fingerprint  # noqa: E402
from paper_1906_10678_amd import synth  # noqa: E402

SCENES = 16
PER_SCENE = 8
MAX_DOF = 6


def queries():
    return synth.queries_c3(oracle.pose_fn_for, scenes=SCENES, per_scene=PER_SCENE)


def solve(args):
    i, q = args
    occ = oracle.raster(q.scene)
    r = oracle.reach(q.arm, occ, q.target, m=(q.arm.dof + 1) // 2 + 1, keep_sets=False)
    return {"query": i, "fingerprint": fingerprint(q), "dof": q.arm.dof, "n": q.scene.n,
            "status": int(r.status), "pose": None if r.pose is None else np.asarray(r.pose).tolist()}


def main():
    oracle.build()
    qs = queries()
    todo = [(i, q) for i, q in enumerate(qs) if q.arm.dof <= MAX_DOF]
    with Pool(min(4, os.cpu_count() or 1)) as p:
        rows = p.map(solve, todo)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_reach.json")
    with open(out, "w") as f:
        json.dump({"scenes": SCENES, "per_scene": PER_SCENE, "max_dof": MAX_DOF, "rows": rows}, f)
    print("wrote", out, len(rows), "queries", [r["status"] for r in rows])


if __name__ == "__main__":
    main()
