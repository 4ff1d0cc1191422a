"""Writes c2_paths.json: the oracle's answers to the 8-DOF reach + 16-waypoint path
queries of seeds 0..15 (status, path, first reach poses in the canonical order), with a
fingerprint of each query's inputs so a stale file is detected.

Only the oracle computes these values (reach at split 6: the answer does not depend on
the split, which the oracle tests pin against brute force).  Run from the repository
root:  python tests/golden/make_c2_paths.py
"""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1906_10678_amd import synth  # noqa: E402

SEEDS = list(range(16))
SPLIT = 6


def fingerprint(q) -> str:
    a, s = q.arm, q.scene
    parts = [a.types, a.lens, a.lo_cdeg, a.hi_cdeg, a.step_cdeg, list(a.base), a.samples,
             s.n, s.dilate, np.asarray(s.boxes).tolist(), np.asarray(s.spheres).tolist(),
             np.asarray(q.start).tolist(), list(q.target), q.waypoints, q.max_delta]
    return hashlib.sha256(json.dumps(parts, default=int).encode()).hexdigest()[:16]


def solve(seed: int):
    q = synth.query_c2(seed, oracle.pose_fn_for)
    occ = oracle.raster(q.scene)
    st, path, res = oracle.plan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, m=SPLIT)
    return {"seed": seed, "fingerprint": fingerprint(q), "status": int(st),
            "path": None if path is None else np.asarray(path).tolist(),
            "reach_poses": [] if res is None else np.asarray(res.sols).tolist()}


def main():
    oracle.build()
    with Pool(min(8, os.cpu_count() or 1)) as p:
        rows = p.map(solve, SEEDS)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_paths.json")
    with open(out, "w") as f:
        json.dump({"split": SPLIT, "queries": rows}, f, indent=1)
    print("wrote", out, [r["status"] for r in rows])


if __name__ == "__main__":
    main()
