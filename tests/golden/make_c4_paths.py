"""Writes c4_paths.json: the oracle's answers to the full-size batched-path plans of
scene 0 (512^3 grid, 8-DOF chain with doubled lengths, 2.5 deg steps) whose waypoint
count is at most 32 (seconds for up to 20 waypoints, up to about 5 minutes and 10 GB
for 21 to 32; far longer for the widest windows), plus the plans listed in EXTRA (of
later scenes), with a fingerprint of each plan's inputs.

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
MAX_W = 32
SPLIT = 5
EXTRA = [(5, 3)]    # (scene, plan index within the scene) of later scenes (27 waypoints)
WORKERS = 3         # memory: the widest windows hold up to about 10 GB each


def plans():
    scenes = 1 + max([sc for sc, _ in EXTRA], default=0)
    return synth.queries_c4(oracle.pose_fn_for, scenes=scenes, per_scene=PLANS)


def solve(args):
    j, q = args
    occ = oracle.raster(q.scene)
    st, path, _ = oracle.plan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, m=SPLIT)
    return {"plan": j, "fingerprint": fingerprint(q), "waypoints": q.waypoints, "status": int(st),
            "path": None if path is None else np.asarray(path).tolist()}


def main():
    oracle.build()
    qs = plans()
    todo = [(j, q) for j, q in enumerate(qs[:PLANS]) if q.waypoints <= MAX_W]
    todo += [(sc * PLANS + j, qs[sc * PLANS + j]) for sc, j in EXTRA]
    todo.sort(key=lambda t: -t[1].waypoints)   # the longest first
    with Pool(min(WORKERS, os.cpu_count() or 1)) as p:
        rows = sorted(p.map(solve, todo, chunksize=1), key=lambda r: r["plan"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_paths.json")
    with open(out, "w") as f:
        json.dump({"split": SPLIT, "plans": PLANS, "max_waypoints": MAX_W, "extra": EXTRA, "rows": rows}, f)
    print("wrote", out, [(r["plan"], r["waypoints"], r["status"]) for r in rows])


if __name__ == "__main__":
    main()
