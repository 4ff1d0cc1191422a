"""Host-core timing of the oracle: the CPU baseline printed beside the GPU figures.

TEST INFRASTRUCTURE ONLY: run by the benchmark's CPU-baseline leg as a child process
(``python -m oracle.timing QUERIES_JSON OUT_JSON PROCS``), never by the GPU library.
It times the oracle as it stands, on the same queries the benchmark solves on the GPU:

* latency: the first query, raster + windowed reach + tube path, on one thread;
* throughput: the first N queries, one per task, over PROCS worker processes (each
  process one thread), wall clock from the first task handed out to the last result.

Table build, raster and the search are all inside the clock (the GPU step also
rasterises its scenes).  Each worker runs with one BLAS/OpenMP thread.
"""
from __future__ import annotations

import json
import os
import sys
import time
from multiprocessing import get_context

import numpy as np


def _arm(d):
    from types import SimpleNamespace

    return SimpleNamespace(**d)


def _scene(d):
    from types import SimpleNamespace

    return SimpleNamespace(n=d["n"], dilate=d["dilate"], boxes=np.asarray(d["boxes"], np.int32).reshape(-1, 6),
                           spheres=np.asarray(d["spheres"], np.int32).reshape(-1, 4))


def solve(d):
    """Raster + plan_path of one serialised query; (seconds, status)."""
    import oracle

    arm, scene = _arm(d["arm"]), _scene(d["scene"])
    t0 = time.perf_counter()
    occ = oracle.raster(scene)
    st, _, _ = oracle.plan_path(arm, occ, np.asarray(d["start"], np.int64), tuple(d["target"]), d["waypoints"],
                                d["max_delta"], m=d["split"], approach=d.get("approach"))
    return time.perf_counter() - t0, int(st)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main(argv):
    src, dst, procs = argv[0], argv[1], int(argv[2])
    with open(src) as f:
        qs = json.load(f)
    import oracle

    oracle.build()
    oracle.lib()
    lat_s, lat_st = solve(qs[0])
    ctx = get_context("fork")
    with ctx.Pool(procs) as pool:
        pool.map(int, range(procs))          # workers up before the clock starts
        t0 = time.perf_counter()
        res = pool.map(solve, qs, chunksize=1)
        wall = time.perf_counter() - t0
    out = {"latency_s": lat_s, "latency_status": lat_st, "throughput_wall_s": wall, "queries": len(qs),
           "procs": procs, "per_query_s": [r[0] for r in res], "statuses": [r[1] for r in res],
           "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}
    with open(dst, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main(sys.argv[1:])
