"""Writes gms_paths.json: the oracle's answers to reach + 16-waypoint path queries of
the two-DOF-per-segment arm (four segments, each a zero-length yaw link and a pitch
joint), seeds 0..7, with a fingerprint of each query's inputs.

Only the oracle computes these values (reach at split 6).  Run from the repository
root:  python tests/golden/make_gms_paths.py
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

SEEDS = list(range(8))
SPLIT = 6


def solve(seed: int):
    q = synth.query_gms(seed, oracle.pose_fn_for)
    occ = oracle.raster(q.scene)
    st, path, res = oracle.plan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, m=SPLIT)
    return {"seed": seed, "fingerprint": fingerprint(q), "status": int(st),
            "path": None if path is None else np.asarray(path).tolist(),
            "reach_poses": [] if res is None else np.asarray(res.sols).tolist()}


def main():
    oracle.build()
    with Pool(min(4, os.cpu_count() or 1)) as p:
        rows = p.map(solve, SEEDS)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gms_paths.json")
    with open(out, "w") as f:
        json.dump({"split": SPLIT, "queries": rows}, f, indent=1)
    print("wrote", out, [r["status"] for r in rows])


if __name__ == "__main__":
    main()
