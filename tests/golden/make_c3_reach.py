"""Writes c3_reach.json: the oracle's answers to full-size batched-reach queries of scenes
0..15 (128^3 / 256^3 grids, unwindowed joints, 5 deg steps), with a fingerprint of each
query's inputs: every query whose arm has at most 6 DOF (seconds each for the oracle),
and the first HIGH_DOF_COUNT queries by index with 7 or 8 DOF (up to about 12 minutes
and 12 GB each).

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
HIGH_DOF_COUNT = 12
WORKERS = 3   # memory: the 8-DOF queries hold up to about 12 GB each


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
    # the long 7-8 DOF queries first, so they overlap with the rest
    todo = [(i, q) for i, q in enumerate(qs) if q.arm.dof > MAX_DOF][:HIGH_DOF_COUNT]
    todo += [(i, q) for i, q in enumerate(qs) if q.arm.dof <= MAX_DOF]
    with Pool(min(WORKERS, os.cpu_count() or 1)) as p:
        rows = sorted(p.map(solve, todo, chunksize=1), key=lambda r: r["query"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_reach.json")
    with open(out, "w") as f:
        json.dump({"scenes": SCENES, "per_scene": PER_SCENE, "max_dof": MAX_DOF, "high_dof_count": HIGH_DOF_COUNT,
                   "rows": rows}, f)
    print("wrote", out, len(rows), "queries", [r["status"] for r in rows])


if __name__ == "__main__":
    main()
