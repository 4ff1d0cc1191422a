"""Benchmark: 8-DOF reach + 16-waypoint path solves on one MI355X.

A step is one whole query of the 256^3 workload: rasterise its scene, run the
windowed staged reach search (tables, orientation sets, forward / backward stage
expansion, compaction, join, D marking, canonical reach pose) and the tube path
search, with the result copied back to the host.  The steps cycle over Q seeded
synthetic queries (scene seeds 0..Q-1), prepared before the timed region.

Prints one JSON line.  `roofline` is for the expansion kernel (the stage
expansions dominate device time): achieved = algorithmic bytes / kernel time, both
summed over the expansion launches of the timed region, the time from HIP events
recorded on the library's stream around each launch; algorithmic bytes per launch
= 8 * (non-zero 64-bit words of the input set + of the output set + occupancy words
of the active box) in the layout [orientation][z][y][x/64].  `cpu_baseline` times
the CPU oracle on one query of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def canonical_words(keys: np.ndarray, n: int, na: int) -> np.ndarray:
    """Word indices of states in the layout [o][z][y][x/64], o = ia*na + ie, from keys
    ((z*n + y)*n + x) << 16 | ia << 8 | ie."""
    keys = np.asarray(keys, np.uint64)
    ie = (keys & np.uint64(0xff)).astype(np.int64)
    ia = ((keys >> np.uint64(8)) & np.uint64(0xff)).astype(np.int64)
    v = (keys >> np.uint64(16)).astype(np.int64)
    x, y, z = v % n, (v // n) % n, v // (n * n)
    wpr = (n + 63) // 64
    o = ia * na + ie
    return np.unique(((o * n + z) * n + y) * wpr + x // 64)


def box_of(keys_list, n):
    lo = np.array([n, n, n])
    hi = np.array([-1, -1, -1])
    for keys in keys_list:
        if len(keys) == 0:
            continue
        v = (np.asarray(keys, np.uint64) >> np.uint64(16)).astype(np.int64)
        xyz = np.stack([v % n, (v // n) % n, v // (n * n)], 1)
        lo = np.minimum(lo, xyz.min(0))
        hi = np.maximum(hi, xyz.max(0))
    return lo, hi


def expansion_bytes(solver, msc, n, na, stats):
    """Algorithmic bytes of every expansion launch of one captured query:
    {(kernel, stage): bytes}."""
    m, dof = stats["split_m"], stats["dof"]
    sets = {}
    for k in range(m + 1):
        sets[("F", k)] = solver.debug_set(msc.SET_F, k)
    for k in range(m, dof + 1):
        sets[("B", k)] = solver.debug_set(msc.SET_B, k)
    out = {}
    wpr = (n + 63) // 64
    for k in range(1, m + 1):
        fin, fout = sets[("F", k - 1)], sets[("F", k)]
        lo, hi = box_of([fin, fout], n)
        occ = 0 if hi[0] < 0 else (hi[2] - lo[2] + 1) * (hi[1] - lo[1] + 1) * (hi[0] // 64 - lo[0] // 64 + 1)
        out[("expand_fwd", k)] = 8 * (len(canonical_words(fin, n, na)) + len(canonical_words(fout, n, na)) + occ)
    for k in range(m, dof):
        bin_, bout = sets[("B", k + 1)], sets[("B", k)]
        lo, hi = box_of([bin_, bout], n)
        occ = 0 if hi[0] < 0 else (hi[2] - lo[2] + 1) * (hi[1] - lo[1] + 1) * (hi[0] // 64 - lo[0] // 64 + 1)
        out[("expand_bwd", k)] = 8 * (len(canonical_words(bin_, n, na)) + len(canonical_words(bout, n, na)) + occ)
    assert wpr >= 1
    return out


def cpu_baseline(queries, split):
    import oracle

    q = queries[0]
    t0 = time.perf_counter()
    occ = oracle.raster(q.scene)
    st, path, _ = oracle.plan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, m=split)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "1 query (scene seed 0): raster + windowed reach (split %d) + tube path, single thread, "
                      "%.1f s, status %d" % (split, dt, st)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--queries", type=int, default=8)
    ap.add_argument("--workspace-gb", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without HIP events (no roofline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    print("preparing %d queries" % args.queries, file=sys.stderr, flush=True)
    queries = [synth.query_c2(s, solver.pose_fn_for) for s in range(args.queries)]
    arm = queries[0].arm
    n, na = queries[0].scene.n, arm.na

    # Algorithmic bytes per expansion launch, from one captured run of each query.
    alg = []
    splits = []
    for q in queries:
        scene = solver.scene(q.scene)
        st, _ = solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta, flags=msc.CAPTURE_SETS)
        stats = solver.stats()
        splits.append(stats["split_m"])
        alg.append(expansion_bytes(solver, msc, n, na, stats))
    print("captured stage sets; splits", splits, file=sys.stderr, flush=True)

    flags = 0 if args.no_profile else msc.PROFILE

    def step(i):
        q = queries[i % len(queries)]
        scene = solver.scene(q.scene)
        st, path = solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta, flags=flags)
        if st != msc.OK:
            raise RuntimeError("query %d: status %d" % (i % len(queries), st))
        return solver.timings() if flags else []

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    lat = []
    launches = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        recs = step(i)
        lat.append(time.perf_counter() - t0)
        launches.append((i % len(queries), recs))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    per_kernel = {}
    for _, recs in launches:
        for kname, stage, nin, nout, ms in recs:
            t = per_kernel.setdefault(kname, [0.0, 0])
            t[0] += ms
            t[1] += 1
    roofline = None
    if launches and launches[0][1]:
        b_sum, ms_sum, cnt = 0.0, 0.0, 0
        for qi, recs in launches:
            for kname, stage, nin, nout, ms in recs:
                if kname in ("expand_fwd", "expand_bwd"):
                    b_sum += alg[qi][(kname, stage)]
                    ms_sum += ms
                    cnt += 1
        achieved = b_sum / (ms_sum * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                    "kernel": "expand (k_expand_fwd + k_expand_bwd)", "launches": cnt,
                    "avg_launch_us": round(1e3 * ms_sum / max(cnt, 1), 2),
                    "alg_bytes_per_launch": round(b_sum / max(cnt, 1))}

    lat_ms = np.array(lat) * 1e3
    result = {
        "metric": "8-DOF reach+path solves/sec",
        "value": round(args.steps / wall, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain single query, reach pose + 16-waypoint path: 8-DOF alternating "
                               "yaw/pitch chain 30,30,25,25,20,20,15,10 voxels, +-170 deg in 5 deg steps, "
                               "256^3 bit-packed grid, dilation 2, 32 boxes + 8 spheres, max 5 deg per joint "
                               "per waypoint; one query per step, scene raster included",
                   "queries": len(queries), "grid": n, "dof": arm.dof, "waypoints": queries[0].waypoints,
                   "splits": splits},
        "roofline": roofline,
        "kernel_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in sorted(per_kernel.items())},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(queries, splits[0])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
