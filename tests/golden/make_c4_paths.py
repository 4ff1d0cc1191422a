"""Writes c4_paths.json: the oracle's answers to the full-size batched-path plans of
scene 0 (512^3 grid, 8-DOF chain with doubled lengths, 2.5 deg steps) whose waypoint
count is at most 20 (the oracle needs seconds for those, far longer for the widest
windows), with a fingerprint of each plan's inputs.

Only the oracle computes these values (reach at split 5).  Run from the repository
root:  python tests/golden/make_c4_paths.py
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

PLANS = 32
MAX_W = 20
SPLIT = 5


def plans():
    return synth.queries_c4(oracle.pose_fn_for, scenes=1, per_scene=PLANS)


def solve(args):
    j, q = args
    occ = oracle.raster(q.scene)
    st, path, _ = oracle.plan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, m=SPLIT)
    return {"plan": j, "fingerprint": fingerprint(q), "waypoints": q.waypoints, "status": int(st),
            "path": None if path is None else np.asarray(path).tolist()}


def main():
    oracle.build()
    qs = plans()
    todo = [(j, q) for j, q in enumerate(qs) if q.waypoints <= MAX_W]
    with Pool(min(4, os.cpu_count() or 1)) as p:
        rows = p.map(solve, todo)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_paths.json")
    with open(out, "w") as f:
        json.dump({"split": SPLIT, "plans": PLANS, "max_waypoints": MAX_W, "rows": rows}, f)
    print("wrote", out, [(r["plan"], r["waypoints"], r["status"]) for r in rows])


if __name__ == "__main__":
    main()
