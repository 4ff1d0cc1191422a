"""Benchmark: 8-DOF reach + 16-waypoint path solves on one MI355X.

A query rasterises its scene, runs the windowed staged reach search (tables,
orientation sets, forward / backward stage expansion, compaction, the meet of the
pathways, D marking, canonical reach pose) and the tube path search, with the result
on the host.  Queries cycle over Q seeded synthetic queries (scene seeds 0..Q-1)
prepared before any timing.

Two phases:
  plain   -- one query per call (msc_path), every launch timed with HIP events on
             the library's stream; gives `plain` and `roofline`;
  batched -- a step is one batch of queries (its scenes rasterised in the step)
             solved by msc_batch over worker lanes; gives `value`, p50/p99 (per
             query, from batch start to completion).

`roofline` is for the stage expansions (k_expand_fwd + k_expand_bwd): achieved =
algorithmic bytes / kernel time summed over the expansion launches of the plain timed
region; algorithmic bytes per launch = 8 * (non-zero 64-bit words of the input set +
of the output set + occupancy words of the active box) in the layout
[orientation][z][y][x/64], from captured stage sets of the same queries.  Also
`copy_GBps` (a 1 GiB device-to-device copy timed in the same run, reads + writes: the
achievable ceiling), `frac_of_copy` = achieved / copy_GBps, and `large_stages`: the
algorithmic rate of the expansion launches above 256 MB (beyond the cache) on full-size
plans, read from the committed summary (profiles/c4_big_stages.md) while the kernel
sources match.
`cpu_baseline` times the CPU oracle on the host cores: all-core throughput over 16 queries of the
same workload (one process per query), with the one-thread latency of query 0 beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
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


def query_record(q, split, approach=None) -> dict:
    """A query as plain JSON for the oracle's timing child."""
    a, sc = q.arm, q.scene
    return {"arm": {"types": list(a.types), "lens": list(a.lens), "lo_cdeg": list(a.lo_cdeg),
                    "hi_cdeg": list(a.hi_cdeg), "step_cdeg": a.step_cdeg, "base": list(a.base),
                    "samples": a.samples, "az0_cdeg": a.az0_cdeg, "el0_cdeg": a.el0_cdeg},
            "scene": {"n": sc.n, "dilate": sc.dilate, "boxes": np.asarray(sc.boxes).tolist(),
                      "spheres": np.asarray(sc.spheres).tolist()},
            "start": np.asarray(q.start).tolist(), "target": list(q.target), "waypoints": q.waypoints,
            "max_delta": q.max_delta, "split": int(split), "approach": list(approach) if approach else None}


def cpu_baseline(queries, splits, approach, procs, count):
    """The oracle on the host cores, in a child process (a fresh interpreter that has not
    touched the GPU): one query on one thread, then `count` queries over `procs` worker
    processes.  value = the all-core throughput."""
    import subprocess
    import tempfile

    procs = max(1, min(procs, len(os.sched_getaffinity(0))))
    count = min(count, len(queries))
    with tempfile.TemporaryDirectory() as tmp:
        src, dst = os.path.join(tmp, "q.json"), os.path.join(tmp, "t.json")
        with open(src, "w") as f:
            json.dump([query_record(queries[i], splits[i], approach) for i in range(count)], f)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        subprocess.run([sys.executable, "-m", "oracle.timing", src, dst, str(procs)], cwd=ROOT, env=env,
                       check=True)
        with open(dst) as f:
            t = json.load(f)
    return {"value": round(t["queries"] / t["throughput_wall_s"], 4), "unit": "solves/s", "cores": t["procs"],
            "kind": "oracle",
            "sample": "%d queries (scene seeds 0..%d) of the same workload, raster + windowed reach + tube path, "
                      "one query per process over %d single-thread processes, %.1f s wall; statuses %s"
                      % (t["queries"], t["queries"] - 1, t["procs"], t["throughput_wall_s"], t["statuses"]),
            "latency_1_thread": {"value": round(1.0 / t["latency_s"], 4), "unit": "solves/s",
                                 "seconds": round(t["latency_s"], 3), "query": 0, "status": t["latency_status"]},
            "nproc": t["nproc"], "affinity_cpus": t["affinity"], "cpu_model": t["cpu_model"]}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "expand_traffic_c2.md")
KERNEL_SOURCES = ["paper_1906_10678_amd/csrc/msc_kernels.hip", "paper_1906_10678_amd/csrc/msc_runtime.hip",
                  "paper_1906_10678_amd/csrc/msc_common.h"]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(field: str = "HBM bytes per expansion launch"):
    """A figure of the committed counter summary (default: HBM bytes per expansion
    launch), or None when the summary is missing, lacks it, or was taken on other kernel
    sources."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel sources sha256") != kernel_source_hash():
        return None
    try:
        return float(fields[field])
    except (KeyError, ValueError):
        return None


def full_size_stages():
    """Algorithmic rate of the expansion launches beyond the cache on full-size plans, from
    the committed summary (profiles/c4_big_stages.md), or None when it is missing or was
    taken on other kernel sources."""
    try:
        with open(C4_STAGES_PROFILE) as f:
            text = f.read()
    except OSError:
        return None
    if "kernel sources sha256: `%s`" % kernel_source_hash() not in text:
        return None
    for line in text.splitlines():
        if line.startswith("- large stages: "):
            parts = line[len("- large stages: "):].split(", ")
            return {"launches": int(parts[0].split()[0]), "alg_GBps": float(parts[1].split()[0]),
                    "frac": float(parts[2].split()[1]), "source": "profiles/c4_big_stages.md"}
    return None


def traffic_run(args):
    """The program that the two rocprofv3 --pmc passes run: captured runs of the C2
    queries (algorithmic bytes per expansion launch), a 1 GiB device copy as the
    counter calibration, then one plain run of each query."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    queries = []
    for s in range(args.queries):
        queries.append(synth.query_c2(s, solver.pose_fn_for))
        print("traffic run: query %d drawn" % s, flush=True)
    n, na = queries[0].scene.n, queries[0].arm.na
    alg_total, launches = 0, 0
    for i, q in enumerate(queries):
        print("traffic run: capturing query %d" % i, flush=True)
        sc = solver.scene(q.scene)
        solver.path(sc, q.arm, q.start, q.target, q.waypoints, q.max_delta, flags=msc.CAPTURE_SETS)
        st = solver.stats()
        a = expansion_bytes(solver, msc, n, na, st)
        used = {k: v for k, v in a.items() if not (k[0] == "expand_fwd" and k[1] == st["split_m"])}
        alg_total += int(sum(used.values()))
        launches += len(used)
    torch.cuda.synchronize()
    x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    for i, q in enumerate(queries):
        print("traffic run: solving query %d" % i, flush=True)
        sc = solver.scene(q.scene)
        solver.path(sc, q.arm, q.start, q.target, q.waypoints, q.max_delta)
    torch.cuda.synchronize()
    out = {"alg_bytes_total": alg_total, "expand_launches": launches, "copy_bytes": 1 << 30,
           "queries": len(queries)}
    os.makedirs(os.path.dirname(args.traffic_out) or ".", exist_ok=True)
    with open(args.traffic_out, "w") as f:
        json.dump(out, f)
    print("traffic run done", json.dumps(out), flush=True)


C4_STAGES_PROFILE = os.path.join(ROOT, "profiles", "c4_big_stages.md")


def c4_stages_run(args):
    """The program of the full-size stage measurement: six batched-path plans (512^3, 2.5
    deg, doubled lengths), each solved once to warm up, a 1 GiB device copy (the counter
    calibration), then each solved once with HIP-event times per launch (the dispatches
    the counter passes are read on), then once more with MSC_COUNT_SETS for the member
    counts and the non-zero words of every stage's output."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    qs = synth.queries_c4(solver.pose_fn_for, scenes=1, per_scene=6)
    scenes = [solver.scene(q.scene) for q in qs]
    for q, sc in zip(qs, scenes):
        solver.path(sc, q.arm, q.start, q.target, q.waypoints, q.max_delta)
    torch.cuda.synchronize()
    x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    plans = []
    for q, sc in zip(qs, scenes):
        st, _ = solver.path(sc, q.arm, q.start, q.target, q.waypoints, q.max_delta, flags=msc.PROFILE)
        stats = solver.stats()
        plans.append({"status": st, "split": stats["split_m"], "waypoints": q.waypoints,
                      "recs": [list(r) for r in solver.timings()]})
        print("c4 stages: plan timed", len(plans), flush=True)
    torch.cuda.synchronize()
    for p, q, sc in zip(plans, qs, scenes):
        st, _ = solver.path(sc, q.arm, q.start, q.target, q.waypoints, q.max_delta,
                            flags=msc.PROFILE | msc.COUNT_SETS)
        recs = solver.timings()
        words = solver.timing_words()
        if [r[0] for r in recs] != [r[0] for r in p["recs"]]:
            raise RuntimeError("the counting run launched other kernels")
        p["out_count"] = [int(r[3]) for r in recs]
        p["out_words"] = words
    torch.cuda.synchronize()
    os.makedirs(os.path.dirname(args.c4_stages_run) or ".", exist_ok=True)
    with open(args.c4_stages_run, "w") as f:
        json.dump({"copy_bytes": 1 << 30, "plans": plans}, f)
    print("c4 stages run done", len(plans), flush=True)


def calibration_copies(dispatches):
    """Dispatch ids of the three 1 GiB calibration copies among (id, kernel name, grid
    size): the copy dispatches of the largest grid (the library's own small uploads and
    the set captures are copies too)."""
    copies = [(i, g) for i, name, g in dispatches if "copyBuffer" in name]
    top = max(g for _, g in copies)
    ids = sorted({i for i, g in copies if g == top})
    if len(ids) != 3:
        raise RuntimeError("expected three calibration copies, found %d" % len(ids))
    return ids


def c4_stages_summary(args):
    """Per expansion launch of the six full-size plans: algorithmic bytes (8 x (input
    states read from the list + non-zero words of the output structure)), HBM bytes (two
    counter passes), the L2 hit rate (a TCC_HIT / TCC_MISS pass) and the HIP-event time of
    a run outside the profiler; the ones above 256 MB algorithmic (beyond the MALL) in a
    table with totals, and the meet's HBM rate."""
    import csv

    fetch_csv, write_csv, tcc_csv, times_json = args.c4_stages_summary
    times = json.load(open(times_json))
    kinds = {"expand_fwd": "k_expand_fwd", "expand_bwd": "k_expand_bwd", "join": "k_"}

    def dispatches(path, counters):
        """Counter values of the timed runs' dispatches after the calibration copies:
        [(kernel name, {counter: value})] in dispatch order."""
        by_id, grid = {}, {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] in counters:
                d = by_id.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], {}])
                d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                grid[int(r["Dispatch_Id"])] = int(r["Grid_Size"])
        ids = sorted(by_id)
        cal_ids = calibration_copies([(i, by_id[i][0], grid[i]) for i in ids])
        last = max(cal_ids)
        return [by_id[i][1] for i in cal_ids], [by_id[i] for i in ids if i > last]

    def set_kernels(rows):
        return [(name, v) for name, v in rows
                if "k_expand_fwd" in name or "k_expand_bwd" in name or "k_meet" in name or "k_join" in name]

    fcal, frows = dispatches(fetch_csv, {"FETCH_SIZE"})
    wcal, wrows = dispatches(write_csv, {"WRITE_SIZE"})
    _, trows = dispatches(tcc_csv, {"TCC_HIT_sum", "TCC_MISS_sum"})
    ff = (times["copy_bytes"] / 1024.0) / (sum(c["FETCH_SIZE"] for c in fcal) / len(fcal))
    wf = (times["copy_bytes"] / 1024.0) / (sum(c["WRITE_SIZE"] for c in wcal) / len(wcal))
    frows, wrows, trows = set_kernels(frows), set_kernels(wrows), set_kernels(trows)
    launches = []
    for i, p in enumerate(times["plans"]):
        for j, r in enumerate(p["recs"]):
            if r[0] in ("expand_fwd", "expand_bwd", "join"):
                launches.append((i, j, r, p["out_words"][j], p["out_count"][j]))
    n = min(len(launches), len(frows), len(wrows), len(trows))
    big, meets, all_exp = [], [], [0.0, 0.0, 0]
    for (i, j, r, words, outc), (fname, fv), (_, wv), (_, tv) in zip(launches[:n], frows, wrows, trows):
        kname = fname.split("(")[0]
        if r[0] == "join" and "k_meet" not in kname and "k_join" not in kname:
            raise RuntimeError("dispatch order does not match the launch records")
        hbm = fv["FETCH_SIZE"] * ff * 1024 + wv["WRITE_SIZE"] * wf * 1024
        hit = tv.get("TCC_HIT_sum", 0.0)
        miss = tv.get("TCC_MISS_sum", 0.0)
        l2 = hit / (hit + miss) if hit + miss > 0 else float("nan")
        ms = r[4]
        if r[0] == "join":
            meets.append((i, kname, r[2], hbm, l2, ms))
            continue
        alg = 8.0 * (r[2] + max(words, 0))
        all_exp[0] += alg
        all_exp[1] += ms
        all_exp[2] += 1
        if alg > 256e6:
            big.append((i, kname, r[1], r[2], words, alg, hbm, l2, ms))
    lines = ["# Full-size plans: expansion stages beyond the cache, against the HBM roofline", "",
             "Six plans of the batched-path workload (512^3 grid, 8-DOF chain with doubled lengths, 2.5 deg).  "
             "Per expansion launch: algorithmic bytes = 8 x (input states, read from the compacted list, + "
             "non-zero 64-bit words of the output set's structure, counted on the device after the launch in a "
             "second solve with MSC_COUNT_SETS); HBM bytes from FETCH_SIZE and WRITE_SIZE passes scaled by a "
             "1 GiB device copy (x %.4f, x %.4f); L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS) from a third "
             "pass; time from HIP events of the timed solve.  The table lists the launches above 256 MB "
             "algorithmic (larger than the MALL), the stages that stream from HBM." % (ff, wf), "",
             "```",
             "python -u bench.py --c4-stages-run gpurun_out/c4_times.json --workspace-gb 200",
             "timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/c4_fetch -o run "
             "-- python -u bench.py --c4-stages-run gpurun_out/c4_pmc.json --workspace-gb 200",
             "timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/c4_write -o run "
             "-- python -u bench.py --c4-stages-run gpurun_out/c4_pmc.json --workspace-gb 200",
             "timeout -s KILL 300 rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --output-format csv -d gpurun_out/c4_tcc "
             "-o run -- python -u bench.py --c4-stages-run gpurun_out/c4_pmc.json --workspace-gb 200",
             "python bench.py --c4-stages-summary gpurun_out/c4_fetch/run_counter_collection.csv "
             "gpurun_out/c4_write/run_counter_collection.csv gpurun_out/c4_tcc/run_counter_collection.csv "
             "gpurun_out/c4_times.json",
             "```", "",
             "| plan | kernel | stage | input states | output words | algorithmic MB | HBM MB | HBM / alg | L2 hit | ms | alg GB/s | of 8 TB/s |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    ta = th = tm = 0.0
    for i, kname, stage, nin, words, alg, hbm, l2, ms in big:
        ta += alg
        th += hbm
        tm += ms
        lines.append("| %d | %s | %d | %d | %d | %.1f | %.1f | %.2f | %.3f | %.3f | %.0f | %.3f |" % (
            i, kname, stage, nin, words, alg / 1e6, hbm / 1e6, hbm / alg, l2, ms, alg / (ms * 1e-3) / 1e9,
            alg / (ms * 1e-3) / 8e12))
    if tm > 0:
        lines.append("| all | %d launches | | | | %.1f | %.1f | %.2f | | %.3f | %.0f | %.3f |" % (
            len(big), ta / 1e6, th / 1e6, th / ta, tm, ta / (tm * 1e-3) / 1e9, ta / (tm * 1e-3) / 8e12))
    lines += ["", "Every expansion launch of the six plans: %d launches, %.1f MB algorithmic in %.3f ms, "
              "%.0f GB/s (%.3f of 8 TB/s)." % (all_exp[2], all_exp[0] / 1e6, all_exp[1],
                                              all_exp[0] / (all_exp[1] * 1e-3) / 1e9 if all_exp[1] else 0,
                                              all_exp[0] / (all_exp[1] * 1e-3) / 8e12 if all_exp[1] else 0), "",
              "The meet (random membership probes into the set of the last backward stage):", "",
              "| plan | input states | HBM MB | L2 hit | ms | HBM GB/s | of 8 TB/s |", "|---|---|---|---|---|---|---|"]
    mh = mm = 0.0
    for i, kname, nin, hbm, l2, ms in meets:
        mh += hbm
        mm += ms
        lines.append("| %d | %d | %.1f | %.3f | %.3f | %.0f | %.3f |" % (
            i, nin, hbm / 1e6, l2, ms, hbm / (ms * 1e-3) / 1e9, hbm / (ms * 1e-3) / 8e12))
    if mm > 0:
        lines.append("| all | | %.1f | | %.3f | %.0f | %.3f |" % (mh / 1e6, mm, mh / (mm * 1e-3) / 1e9,
                                                                 mh / (mm * 1e-3) / 8e12))
    lines += ["", "- large stages: %d launches, %.0f GB/s algorithmic, frac %.4f" % (
        len(big), ta / (tm * 1e-3) / 1e9 if tm else 0, ta / (tm * 1e-3) / 8e12 if tm else 0),
        "- kernel sources sha256: `%s`" % kernel_source_hash(), ""]
    with open(C4_STAGES_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("wrote", C4_STAGES_PROFILE, flush=True)


def traffic_summary(args):
    """Writes the expansion-traffic summary from the two counter CSVs of the traffic run."""
    import csv
    import collections

    if len(args.traffic_summary) not in (3, 4):
        raise SystemExit("--traffic-summary takes FETCH_CSV WRITE_CSV ALG_JSON [TCC_CSV]")
    fetch_csv, write_csv, alg_json = args.traffic_summary[:3]
    tcc_csv = args.traffic_summary[3] if len(args.traffic_summary) == 4 else None
    alg = json.load(open(alg_json))

    def per_kernel(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        cal_ids = calibration_copies([(int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"])) for r in rows])
        last = max(cal_ids)
        cal = [float(r["Counter_Value"]) for r in rows if int(r["Dispatch_Id"]) in cal_ids]
        per = collections.defaultdict(lambda: [0.0, 0])
        for r in rows:
            if int(r["Dispatch_Id"]) > last:
                name = r["Kernel_Name"].split("(")[0]
                per[name][0] += float(r["Counter_Value"])
                per[name][1] += 1
        return (alg["copy_bytes"] / 1024.0) / (sum(cal) / len(cal)), per

    ff, fper = per_kernel(fetch_csv, "FETCH_SIZE")
    wf, wper = per_kernel(write_csv, "WRITE_SIZE")
    hper = mper = None
    if tcc_csv:
        _, hper = per_kernel(tcc_csv, "TCC_HIT_sum")
        _, mper = per_kernel(tcc_csv, "TCC_MISS_sum")
    expand = [k for k in fper if is_expansion(k)]
    tot = sum(fper[k][0] * ff * 1024 + wper[k][0] * wf * 1024 for k in expand)
    nl = sum(fper[k][1] for k in expand)
    lines = ["# HBM traffic of the stage expansions, 8-DOF reach + path workload (%d queries)" % alg["queries"], "",
             "Three rocprofv3 counter passes over the same program (`bench.py --traffic-run`):", "",
             "```", "timeout -s KILL 420 rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o run "
             "-- python -u bench.py --traffic-run --queries 16",
             "timeout -s KILL 420 rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o run "
             "-- python -u bench.py --traffic-run --queries 16",
             "timeout -s KILL 420 rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --output-format csv "
             "-d gpurun_out/pmc_tcc -o run -- python -u bench.py --traffic-run --queries 16",
             "python bench.py --traffic-summary gpurun_out/pmc_fetch/run_counter_collection.csv "
             "gpurun_out/pmc_write/run_counter_collection.csv gpurun_out/traffic_alg.json "
             "gpurun_out/pmc_tcc/run_counter_collection.csv", "```", "",
             "Counters are KiB per dispatch.  Calibration: a 1 GiB device-to-device copy reads "
             "%.4f x its FETCH_SIZE and writes %.4f x its WRITE_SIZE; both factors are applied." % (ff, wf), "",
             "| kernel | dispatches | fetch MB | write MB | L2 requests (10^6) | L2 hit rate |",
             "|---|---|---|---|---|---|"]
    for k in sorted(set(fper) | set(wper)):
        l2 = "| - | - |"
        if hper is not None and k in hper:
            req = hper[k][0] + mper[k][0]
            l2 = "| %.2f | %.3f |" % (req / 1e6, hper[k][0] / req if req else 0.0)
        lines.append("| %s | %d | %.1f | %.1f %s" % (k, fper[k][1], fper[k][0] * ff * 1024 / 1e6,
                                                      wper[k][0] * wf * 1024 / 1e6, l2))
    lines += ["", "- expansion launches: %d (algorithmic record: %d)" % (nl, alg["expand_launches"]),
              "- algorithmic bytes per expansion launch: %.0f" % (alg["alg_bytes_total"] / alg["expand_launches"]),
              "- HBM bytes per expansion launch: %.0f" % (tot / max(nl, 1)),
              ] + ([] if hper is None else [
              "- L2 requests per expansion launch: %.0f" % (sum(hper[k][0] + mper[k][0] for k in expand) / max(nl, 1)),
              "- L2 hit rate of the expansions: %.3f" % (sum(hper[k][0] for k in expand) /
                                                        max(1.0, sum(hper[k][0] + mper[k][0] for k in expand)))]) + [
              "- kernel sources sha256: `%s`" % kernel_source_hash(), ""]
    with open(TRAFFIC_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("wrote", TRAFFIC_PROFILE, flush=True)


GMS_PROFILE = os.path.join(ROOT, "profiles", "gap_search_2deg.md")


def gms_summary(args):
    """Writes the gap search's kernel summary from rocprofv3's kernel statistics of a
    `--workload gms` run and the JSON line that run printed."""
    import csv

    stats_csv, bench_json = args.gms_summary
    res = None
    for line in open(bench_json):
        line = line.strip()
        if line.startswith("{"):
            res = json.loads(line)
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# Gap search (the paper's quiver method), 2 degree quiver on the 8-DOF workload's scenes", "",
             "```", "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_gms -o run "
             "-- python -u bench.py --workload gms --queries %d --plain-steps %d" % (res["queries"], args.plain_steps),
             "python bench.py --gms-summary gpurun_out/prof_gms/run_kernel_stats.csv gpurun_out/gms_bench.json",
             "```", "",
             "%s.  Each step solves one target with every solution counted (msc_gms_reach), then "
             "again searching only until the first 8 are known (msc_gms_reach_first)." % res["config"]["workload"], "",
             "- solutions per target: %s" % res["solutions"],
             "- every solution counted, in the profiled run: %.1f solves/s, p50 %.2f ms, p99 %.2f ms"
             % (res["all_solutions"]["solves_per_s"], res["all_solutions"]["p50_ms"], res["all_solutions"]["p99_ms"]),
             "- first 8 solutions, in the profiled run: %.1f solves/s, p50 %.2f ms, p99 %.2f ms"
             % (res["first_8_solutions"]["solves_per_s"], res["first_8_solutions"]["p50_ms"],
                res["first_8_solutions"]["p99_ms"]),
             "- kernel sources sha256: `%s`" % kernel_source_hash(), "",
             "| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        lines.append("| %s | %s | %.2f | %.1f | %.1f %% |" % (r["Name"].split("(")[0], r["Calls"],
                                                               float(r["TotalDurationNs"]) / 1e6,
                                                               float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    lines.append("")
    with open(GMS_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("wrote", GMS_PROFILE, flush=True)


TRACE_PROFILE = os.path.join(ROOT, "profiles", "expand_trace_c2.md")


def is_expansion(kernel_name: str) -> bool:
    """The stage-expansion kernels (forward, backward, backward into a hash set), whatever
    their template arguments."""
    name = kernel_name.split("(")[0]
    return any(k in name for k in ("k_expand_fwd", "k_expand_bwd"))


def trace_summary(args):
    """Kernel-trace summary of a --plain-only run, restricted to the plain timed region
    (the last `plain_steps` queries; each starts with its start-pose check): per-kernel
    statistics, and the average duration of the expansion dispatches of the queries the
    roofline counts (those with algorithmic bytes), next to the HIP-event average of the
    same launches that the run printed."""
    import csv
    import collections

    trace_csv, bench_json = args.trace_summary
    res = None
    for line in open(bench_json):
        line = line.strip()
        if line.startswith("{"):
            res = json.loads(line)
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if "k_pose_check" in r["Kernel_Name"]][-args.plain_steps:]
    nq, n_alg = res["queries"], res["roofline"]["alg_queries"]
    timed = rows[starts[0]:]
    t_first = int(rows[starts[0]]["Start_Timestamp"])
    tail = []
    for s_idx, a in enumerate(starts):
        b = starts[s_idx + 1] if s_idx + 1 < len(starts) else len(rows)
        if s_idx % nq < n_alg:
            tail += [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows[a:b]
                     if is_expansion(r["Kernel_Name"])]
    nl = len(tail)
    stats = collections.defaultdict(list)
    for r in timed:
        stats[r["Kernel_Name"].split("(")[0]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["# Kernel trace, 8-DOF reach + 16-waypoint path queries (plain phase of bench.py)", "",
             "```", "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof -o run "
             "-- python -u bench.py --plain-only --no-cpu-baseline",
             "python bench.py --trace-summary gpurun_out/prof/run_kernel_trace.csv gpurun_out/prof_bench.json", "```", "",
             "The run captures the stage sets of the first %d of its %d queries (algorithmic bytes), warms up, "
             "then times %d plain queries (query i %% %d); the roofline's launches are the expansion dispatches "
             "of the timed queries with algorithmic bytes." % (n_alg, nq, args.plain_steps, nq), "",
             "- expansion dispatches counted: %d (the run's HIP-event record: %d)" % (nl, res["roofline"]["launches"]),
             "- their average duration, kernel trace (us): %.2f" % (sum(tail) / max(len(tail), 1)),
             "- their average duration, HIP events in the run (us): %.2f" % res["roofline"]["avg_launch_us"],
             "- algorithmic bytes per expansion launch: %d" % res["roofline"]["alg_bytes_per_launch"],
             "- plain solves/s in the traced run: %.1f" % res["plain"]["solves_per_s"],
             "- kernel sources sha256: `%s`" % kernel_source_hash(), "",
             "Per-kernel statistics of the timed region (%d dispatches, %.1f ms from its first expansion "
             "dispatch to the end of the run):" % (len(timed), (int(timed[-1]["End_Timestamp"]) - t_first) / 1e6), "",
             "| kernel | calls | total ms | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| %s | %d | %.2f | %.1f | %.1f | %.1f |" % (k, len(v), sum(v) / 1e3, sum(v) / len(v), min(v),
                                                               max(v)))
    lines.append("")
    with open(TRACE_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("wrote", TRACE_PROFILE, flush=True)


def serve_poisson(solver, msc, queries, scenes, rate, seconds, rng):
    """Queries submitted to the running server as a Poisson stream of the given rate for
    `seconds`, cycling over `queries`; latency from submission to completion, measured by
    the library.  Returns a row of served/s, p50/p99 and status counts."""
    gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 8)
    t_arr = np.cumsum(gaps)
    t_arr = t_arr[t_arr < seconds]
    pending, lat, sts = [], [], []
    t0 = time.perf_counter()
    i = 0
    while i < len(t_arr) or pending:
        now = time.perf_counter() - t0
        while i < len(t_arr) and t_arr[i] <= now:
            q = queries[i % len(queries)]
            spec = msc.QuerySpec(scenes[i % len(queries)], q.arm, q.target, start=q.start,
                                 waypoints=q.waypoints, delta=q.max_delta)
            pending.append((solver.submit(spec), spec))
            i += 1
        still = []
        for t, spec in pending:
            if solver.poll(t):
                st, _, ms = spec.result()
                lat.append(ms)
                sts.append(st)
            else:
                still.append((t, spec))
        pending = still
        if i < len(t_arr) and not pending:
            time.sleep(max(0.0, min(0.001, t_arr[i] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    return {"offered_per_s": rate, "served": len(lat), "served_per_s": round(len(lat) / wall, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "statuses": {str(k): sts.count(k) for k in sorted(set(sts))}}


def bench_c2serve(args):
    """The 8-DOF reach + path queries arriving as a Poisson stream, served by the server
    with one lane (one query at a time: the plain form) and with several lanes (queries
    overlap on the device): served/s and p50/p99 latency from submission to completion
    at each offered rate."""
    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    queries = [synth.query_c2(s, solver.pose_fn_for) for s in range(args.queries)]
    scenes = [solver.scene(q.scene) for q in queries]
    rng = np.random.default_rng(7)
    out_rows = []
    for lanes in (1, args.lanes if args.lanes > 0 else 8):
        solver.set_lanes(lanes)
        solver.server_start()
        try:
            for rate in args.serve_rates:
                row = {"lanes": lanes}
                row.update(serve_poisson(solver, msc, queries, scenes, rate, args.serve_seconds, rng))
                out_rows.append(row)
                print(json.dumps(row), file=sys.stderr, flush=True)
        finally:
            solver.server_stop()
    solver.set_lanes(0)
    print(json.dumps({"metric": "8-DOF reach+path served/s and p50/p99 ms under Poisson arrivals",
                      "seconds_per_rate": args.serve_seconds, "rows": out_rows,
                      "config": {"workload": "the %d 8-DOF reach + 16-waypoint path queries of the benchmark, "
                                             "Poisson arrivals, latency from submission to completion; one lane "
                                             "= one query at a time" % len(queries)}}), flush=True)


def bench_c3(args):
    """Batched reach poses: 64 scenes (128^3 or 256^3, 10..60 boxes), 8 queries each, DOF
    5..8 unwindowed (+-170 deg in 5 deg steps); targets are ends of random poses, so
    some have no answer.  All queries in one msc_batch call per step."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    qs = synth.queries_c3(solver.pose_fn_for, scenes=args.c3_scenes, per_scene=8)
    print("c3: %d queries" % len(qs), file=sys.stderr, flush=True)

    def step():
        scenes, specs = {}, []
        for q in qs:
            if id(q.scene) not in scenes:
                scenes[id(q.scene)] = solver.scene(q.scene)
            specs.append(msc.QuerySpec(scenes[id(q.scene)], q.arm, q.target))
        return solver.batch(specs)

    tuned = None
    if args.autotune and args.autotune != "none":
        # launch shapes tuned on the first 32 queries (a cache of its own: other sizes)
        cache = args.autotune.replace("msc_tune_c2", "msc_tune_c3")
        ts = time.perf_counter()
        scenes = {}
        specs = []
        for q in qs[:32]:
            if id(q.scene) not in scenes:
                scenes[id(q.scene)] = solver.scene(q.scene)
            specs.append(msc.QuerySpec(scenes[id(q.scene)], q.arm, q.target))
        entries = solver.autotune(specs, cache)
        tuned = {"entries": len(entries), "non_default": sum(1 for e in entries if e[2] != 0),
                 "seconds": round(time.perf_counter() - ts, 2), "cache": cache}
        print("autotune", tuned, file=sys.stderr, flush=True)
    lanes = args.lanes if args.lanes > 0 else 8
    solver.set_lanes(lanes)
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sts = [r[0] for r in res]
    lat = np.array([r[2] for r in res])
    out = {"metric": "batched reach solves/sec", "value": round(args.steps * len(qs) / wall, 3), "unit": "solves/s",
           "steps": args.steps, "ms_per_step": round(1e3 * wall / args.steps, 3), "lanes": lanes,
           "queries": len(qs), "solved_fraction": round(sts.count(msc.OK) / len(sts), 4),
           "statuses": {str(k): sts.count(k) for k in set(sts)},
           "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "autotune": tuned,
           "config": {"workload": "batched reach: 64 scenes 128^3/256^3, 8 queries each, DOF 5..8, unwindowed, 5 deg"}}
    print(json.dumps(out), flush=True)


def bench_c4(args):
    """Batched paths at full size: 8 scenes of 512^3 (40 boxes + 16 spheres, dilation 4),
    32 plans each, 8-DOF chain with doubled segment lengths, 2.5 deg steps (144 bins),
    8..64 waypoints of at most one step per joint.  All 256 plans in msc_batch calls over
    worker lanes that split a large workspace (memory per plan reaches tens of GB)."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    qs = synth.queries_c4(solver.pose_fn_for, scenes=args.c4_scenes, per_scene=32)
    print("c4: %d plans" % len(qs), file=sys.stderr, flush=True)
    scenes = {}
    specs = []
    for q in qs:
        key = q.seed[:2]
        if key not in scenes:
            scenes[key] = solver.scene(q.scene)
        specs.append(msc.QuerySpec(scenes[key], q.arm, q.target, start=q.start, waypoints=q.waypoints,
                                   delta=q.max_delta))
    lanes = args.lanes if args.lanes > 0 else 4
    solver.set_lanes(lanes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = solver.batch(specs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sts = [r[0] for r in res]
    lat = np.array([r[2] for r in res])
    out = {"metric": "batched 8-DOF path plans/sec (512^3, 2.5 deg)", "value": round(len(qs) / wall, 3),
           "unit": "plans/s", "seconds": round(wall, 3), "lanes": lanes, "plans": len(qs),
           "workspace_gb": args.workspace_gb, "statuses": {str(k): sts.count(k) for k in sorted(set(sts))},
           "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "no_path_plans": [[i, qs[i].waypoints] for i, st in enumerate(sts) if st == msc.NO_PATH],
           "config": {"workload": "batched paths: 8 scenes 512^3 (40 boxes + 16 spheres, dilation 4), 32 plans "
                                  "each, 8-DOF doubled lengths, 2.5 deg, 8..64 waypoints"}}
    print(json.dumps(out), flush=True)


def bench_refine(args):
    """Exact end points (msc_refine) of 2^20 discrete poses of the two-DOF-per-segment arm,
    each with a target point inside its end voxel: whole-call rate (host arrays in and
    out) and the kernel's own time from its HIP events; the oracle on a sample."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    arm = synth.arm_gms()
    count = 1 << 20
    rng = synth.rng_for(912, 0)
    q = synth.candidate_poses(rng, arm, count)
    empty = synth.Scene(n=512, dilate=0, boxes=np.zeros((0, 6), np.int32), spheres=np.zeros((0, 4), np.int32))
    scene = solver.scene(empty)
    _, ends = solver.pose_check(scene, arm, q)
    targets = ends.astype(np.float64) + rng.uniform(-0.5, 0.5, size=(count, 3))
    solver.refine(arm, q[:4096], targets[:4096])
    torch.cuda.synchronize()
    walls, kern = [], []
    for _ in range(max(1, args.steps)):
        t0 = time.perf_counter()
        ang, st = solver.refine(arm, q, targets)
        walls.append(time.perf_counter() - t0)
        kern.append(sum(r[4] for r in solver.timings() if r[0] == "refine"))
    wall, kms = float(np.median(walls)), float(np.median(kern))
    # FP64 bytes per pose: 8 int32 angles + 3 doubles in, 8 doubles + 1 int32 out
    bytes_per_pose = arm.dof * 4 + 24 + arm.dof * 8 + 4
    out = {"metric": "exact end points/sec (two-DOF-per-segment arm, FP64)", "value": round(count / wall, 1),
           "unit": "poses/s", "poses": count, "refined": int((st == 0).sum()),
           "kernel_ms": round(kms, 4), "kernel_poses_per_s": round(count / (kms * 1e-3), 1),
           "kernel_GBps": round(count * bytes_per_pose / (kms * 1e-3) / 1e9, 2),
           "config": {"workload": "2^20 uniform poses of the 4 x 2-DOF arm, targets uniform in the end voxel; "
                                  "value includes the host-device copies"}}
    if not args.no_cpu_baseline:
        import oracle
        k = 2000
        t0 = time.perf_counter()
        for i in range(k):
            oracle.refine(arm, q[i], targets[i])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(k / dt, 1), "unit": "poses/s", "cores": 1, "kind": "oracle",
                               "sample": "first %d poses, single thread" % k}
    print(json.dumps(out), flush=True)


def bench_replan(args):
    """Midcourse replanning (msc_replan) on the 16 8-DOF queries: each with a reference
    path, the straight 16-move line from the start toward a drawn pose of the window;
    one replan per call, every reach pose of the first four tried and the path nearest
    the reference kept."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    queries = [synth.query_c2(s, solver.pose_fn_for) for s in range(args.queries)]
    refs = []
    for i, q in enumerate(queries):
        rng = synth.rng_for(916, i)
        goal = np.asarray(q.start, np.int64) + rng.integers(-16, 17, size=q.arm.dof)
        refs.append(np.rint(np.linspace(q.start, goal, q.waypoints + 1)).astype(np.int64))
    scenes = [solver.scene(q.scene) for q in queries]
    statuses, picks = {}, {}
    for i, q in enumerate(queries):
        st, _ = solver.replan(scenes[i], q.arm, q.start, q.target, q.waypoints, q.max_delta, refs[i])
        statuses[i] = st
        picks[i] = solver.stats()["reach_index"] if st == msc.OK else -1
    torch.cuda.synchronize()
    lat, kern = [], []
    t0 = time.perf_counter()
    for k in range(args.plain_steps):
        i = k % len(queries)
        q = queries[i]
        ts = time.perf_counter()
        st, _ = solver.replan(scenes[i], q.arm, q.start, q.target, q.waypoints, q.max_delta, refs[i],
                              flags=msc.PROFILE)
        lat.append(time.perf_counter() - ts)
        kern.append(sum(r[4] for r in solver.timings()))
        if st != statuses[i]:
            raise RuntimeError("replan %d: status %d, first run %d" % (i, st, statuses[i]))
    wall = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    out = {"metric": "8-DOF replans/sec (nearest of the first four reach poses' paths)",
           "value": round(args.plain_steps / wall, 3), "unit": "replans/s",
           "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
           "gpu_ms_per_replan": round(float(np.mean(kern)), 4),
           "statuses": [statuses[i] for i in range(len(queries))],
           "chosen_reach_pose": [picks[i] for i in range(len(queries))],
           "config": {"workload": "the 16 8-DOF reach + 16-waypoint path queries, each with a straight reference "
                                  "path toward a drawn pose; one replan per call"}}
    if args.cpu_replan:
        # about two minutes of single-thread oracle work (radius-2 tube searches in numpy)
        import oracle
        q = queries[0]
        t0 = time.perf_counter()
        occ = oracle.raster(q.scene)
        oracle.replan_path(q.arm, occ, q.start, q.target, q.waypoints, q.max_delta, refs[0])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "replans/s", "cores": 1, "kind": "oracle",
                               "sample": "query 0, single thread, %.1f s" % dt}
    print(json.dumps(out), flush=True)


def bench_guided(args):
    """Workspace-guided paths on the 8-DOF workload's scenes: reach-pose-guided paths to
    the queries' targets (--workload guided), or paths from their start poses to their
    targets through a virtual arm of three 20-voxel segments (--workload posepath).  One
    query per call (every launch timed with HIP events), then batches over worker lanes
    with the tracking on each lane and fused into one launch per batch."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    nq = args.queries
    queries = [synth.query_c2(s, solver.pose_fn_for) for s in range(nq)]
    scenes = [solver.scene(q.scene) for q in queries]
    varm = synth.arm_virtual([20, 20, 20])
    kind = 2 if args.workload == "guided" else 3

    def alone(i, flags=0):
        q = queries[i]
        if kind == 2:
            return solver.guided_path(scenes[i], q.arm, q.target, flags=flags)
        return solver.pose_path(scenes[i], q.arm, q.start, q.target, varm, flags=flags)

    def spec(i):
        q = queries[i]
        if kind == 2:
            return msc.QuerySpec(scenes[i], q.arm, q.target, kind=2)
        return msc.QuerySpec(scenes[i], q.arm, q.target, start=q.start, kind=3, virtual_arm=varm)

    first = [alone(i) for i in range(nq)]
    statuses = [st for st, _ in first]
    rows = [0 if r is None else len(r) for _, r in first]
    torch.cuda.synchronize()
    lat, per_kernel = [], {}
    t0 = time.perf_counter()
    for i in range(args.plain_steps):
        ts = time.perf_counter()
        st, _ = alone(i % nq, msc.PROFILE)
        lat.append(time.perf_counter() - ts)
        if st != statuses[i % nq]:
            raise RuntimeError("query %d: status %d, first run %d" % (i % nq, st, statuses[i % nq]))
        for kname, stage, nin, nout, ms in solver.timings():
            t = per_kernel.setdefault(kname, [0.0, 0])
            t[0] += ms
            t[1] += 1
    wall = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    plain = {"solves_per_s": round(args.plain_steps / wall, 3), "p50_ms": round(float(np.percentile(lat, 50)), 4),
             "p99_ms": round(float(np.percentile(lat, 99)), 4),
             "kernel_ms_per_query": {k: round(v[0] / args.plain_steps, 4) for k, v in sorted(per_kernel.items())}}
    print("plain", plain, file=sys.stderr, flush=True)
    lanes = args.lanes if args.lanes > 0 else 12
    solver.set_lanes(lanes)
    batched = {}
    try:
        for name, flags in (("per_lane", 0), ("fused", msc.FUSED_TRACK)):
            def step():
                specs = [spec(i) for i in range(nq)]
                res = solver.batch(specs, flags=flags)
                for i, (st, r, _) in enumerate(res):
                    if st != statuses[i] or (st == msc.OK and not np.array_equal(r, first[i][1])):
                        raise RuntimeError("batched query %d differs from alone" % i)
                return [r[2] for r in res]
            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            ql = []
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ql.extend(step())
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            ql = np.array(ql)
            batched[name] = {"solves_per_s": round(args.steps * nq / w, 3),
                             "p50_ms": round(float(np.percentile(ql, 50)), 4),
                             "p99_ms": round(float(np.percentile(ql, 99)), 4)}
            print(name, batched[name], file=sys.stderr, flush=True)
    finally:
        solver.set_lanes(0)
    what = ("reach-pose-guided paths (joint 6 of 8 walks the reach pose's samples back to the end of segment 1)"
            if kind == 2 else "paths from the start pose through a virtual arm of three 20-voxel segments "
                              "(end effector tracked)")
    print(json.dumps({"metric": "8-DOF workspace-guided path solves/sec and p50/p99 ms", "workload": args.workload,
                      "queries": nq, "statuses": statuses, "rows": rows, "plain": plain, "batched": batched,
                      "lanes": lanes, "batch": nq,
                      "config": {"workload": "%s; the 8-DOF path workload's scenes and targets (256^3, 5 deg), "
                                             "filter one step, relaxed two, tolerance 3 voxels" % what}}),
          flush=True)


def bench_short(args):
    """Short reaches on the 8-DOF workload's scenes: targets at the middle sample of
    segment 3 or 4 of a drawn valid pose (reachable by a sublength of the arm), solved
    with msc_short_path (hit radius 2 voxels, segments 2..4), one query per call."""
    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    nq = args.queries
    items = []
    for sd in range(nq):
        q = synth.query_c2(sd, solver.pose_fn_for)
        scene = solver.scene(q.scene)
        rng = synth.rng_for(12, sd, 0)
        start, _, _ = synth.first_valid_pose(rng, q.arm, solver.pose_fn_for(q.arm, q.scene))
        seg = 2 + sd % 2          # 0-based: segment 3 or 4
        # about the middle of that segment: the end of the prefix with the segment halved,
        # replayed by the library
        half = synth.Arm(types=q.arm.types[:seg + 1], lens=q.arm.lens[:seg] + [q.arm.lens[seg] // 2],
                         lo_cdeg=q.arm.lo_cdeg[:seg + 1], hi_cdeg=q.arm.hi_cdeg[:seg + 1],
                         step_cdeg=q.arm.step_cdeg, base=q.arm.base)
        _, t = solver.pose_check(scene, half, start[None, :seg + 1])
        items.append((scene, q.arm, tuple(int(v) for v in t[0])))
    first = [solver.short_path(sc, arm, t, 4, 4) for sc, arm, t in items]
    torch.cuda.synchronize()
    lat, per_kernel = [], {}
    t0 = time.perf_counter()
    for i in range(args.plain_steps):
        sc, arm, t = items[i % nq]
        ts = time.perf_counter()
        st, _, _ = solver.short_path(sc, arm, t, 4, 4, flags=msc.PROFILE)
        lat.append(time.perf_counter() - ts)
        if st != first[i % nq][0]:
            raise RuntimeError("query %d: status changed" % (i % nq))
        for kname, stage, nin, nout, ms in solver.timings():
            v = per_kernel.setdefault(kname, [0.0, 0])
            v[0] += ms
            v[1] += 1
    wall = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    print(json.dumps({"metric": "8-DOF short-reach path solves/sec and p50/p99 ms", "queries": nq,
                      "statuses": [f[0] for f in first], "hits": [None if f[2] is None else f[2]["k"] for f in first],
                      "rows": [0 if f[1] is None else len(f[1]) for f in first],
                      "solves_per_s": round(args.plain_steps / wall, 3),
                      "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
                      "kernel_ms_per_query": {k: round(v[0] / args.plain_steps, 4) for k, v in sorted(per_kernel.items())},
                      "config": {"workload": "8-DOF path workload scenes; target at the middle of segment 3 or 4 of a "
                                             "drawn valid pose; hit radius 2 voxels over segments 2..4"}}), flush=True)


def bench_gms(args):
    """The paper's own search (the gap search: 2 degree quiver, about 10^4 vectors;
    segments 1, 2 and 4 from the quiver, segment 3 the free vector across the gap) on the
    8-DOF workload's 256^3 scenes and targets: one query per call, first with every
    solution counted (msc_gms_reach), then searching only until the first 8 in order are
    found (msc_gms_reach_first); both return the same first 8."""
    import torch

    from paper_1906_10678_amd import msc, synth

    class Arm:
        lens = [60.0, 50.0, 40.0, 25.0]
        base = (128, 128, 0)
        step_cdeg, m_min, samples, seg1_min_el_cdeg = 200, 4, 8, 0
        max_flex_cdeg = (12000, 12000, 12000)
        approach = (0, -9000, 4500)
        eps = 0.5

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    nq = args.queries
    items = []
    for sd in range(nq):
        q = synth.query_c2(sd, solver.pose_fn_for)
        items.append((solver.scene(q.scene), q.target))
    first = [solver.gms_reach(sc, Arm, t, 8) for sc, t in items]
    torch.cuda.synchronize()

    def timed(first_only):
        lat = []
        t0 = time.perf_counter()
        for i in range(args.plain_steps):
            sc, t = items[i % nq]
            ts = time.perf_counter()
            st, cnt, sols, _ = solver.gms_reach(sc, Arm, t, 8, first_only=first_only)
            lat.append(time.perf_counter() - ts)
            ref = first[i % nq]
            if st != ref[0] or not np.array_equal(sols, ref[2]) or (not first_only and cnt != ref[1]):
                raise RuntimeError("query %d: answer changed" % (i % nq))
        wall = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        return {"solves_per_s": round(args.plain_steps / wall, 3), "p50_ms": round(float(np.percentile(lat, 50)), 4),
                "p99_ms": round(float(np.percentile(lat, 99)), 4)}

    every = timed(False)
    print("gms all solutions", every, file=sys.stderr, flush=True)
    firsts = timed(True)
    print(json.dumps({"metric": "gap-search reach solves/sec and p50/p99 ms (paper's quiver method)", "queries": nq,
                      "statuses": [f[0] for f in first], "solutions": [f[1] for f in first],
                      "all_solutions": every, "first_8_solutions": firsts,
                      "config": {"workload": "2 deg quiver (10313 vectors), segments 60/50/40/25 voxels, flexion limits "
                                             "120 deg, approach cone 45 deg around straight down, eps 0.5 voxel, "
                                             "8-DOF path workload scenes and targets (256^3)"}}), flush=True)


def bench_c5(args):
    """Serving with dynamic obstacles: Poisson arrivals, 70% reach / 30% path, moving
    boxes re-rasterised every 10 ms tick, midcourse replanning; p50/p99 per class."""
    from paper_1906_10678_amd import msc, serve

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    lanes = args.lanes if args.lanes > 0 else 8
    solver.set_lanes(lanes)
    rows = []
    for rate in args.c5_rates:
        loop = serve.ServingLoop(solver, nscenes=16, seed=0, rate=rate, templates=args.c5_templates,
                                 max_pending=args.c5_max_pending)
        rep = loop.run(seconds=args.c5_seconds, warmup_s=1.0)
        row = {"rate_per_s": rate}
        row.update(rep.summary())
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    out = {"metric": "served solves/sec and p50/p99 ms", "lanes": lanes, "seconds": args.c5_seconds,
           "max_pending": args.c5_max_pending, "rows": rows,
           "config": {"workload": "serving: 16 scenes 256^3 + 1..8 moving boxes, 70% reach / 30% path (8..32 "
                                  "waypoints), DOF 6..8, 10 ms ticks, replans on collision"}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--c4-stages-run", metavar="OUT_JSON",
                    help="run the program of the full-size big-stage measurement (see profiles/c4_big_stages.md)")
    ap.add_argument("--c4-stages-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "TCC_CSV", "TIMES_JSON"),
                    help="write profiles/c4_big_stages.md")
    ap.add_argument("--arm", choices=["chain", "gms"], default="chain",
                    help="gms: the same workload with the paper's arm model, two DOF per segment (a variant)")
    ap.add_argument("--workload", choices=["c2", "c2serve", "c3", "c4", "c5", "refine", "replan", "guided",
                                           "posepath", "short", "gms"], default="c2",
                    help="c2: 8-DOF reach + path (default); c2serve: the same queries served under Poisson "
                         "arrivals, one lane vs several; c3: batched reach; c4: batched paths at 512^3; "
                         "c5: serving with moving obstacles")
    ap.add_argument("--c4-scenes", type=int, default=8)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[200.0, 400.0, 600.0, 900.0])
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--c3-scenes", type=int, default=64)
    ap.add_argument("--c5-rates", type=float, nargs="+", default=[200.0, 500.0, 1000.0, 2000.0])
    ap.add_argument("--c5-seconds", type=float, default=10.0)
    ap.add_argument("--c5-templates", type=int, default=3000)
    ap.add_argument("--c5-max-pending", type=int, default=32,
                    help="serving: the server refuses requests while this many wait for a lane (0: no limit)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed batches")
    ap.add_argument("--warmup", type=int, default=2, help="untimed batches")
    ap.add_argument("--batch", type=int, default=64, help="queries per batch")
    ap.add_argument("--lanes", type=int, default=0, help="worker lanes (0: pick the best of a short sweep)")
    ap.add_argument("--queries", type=int, default=64,
                    help="distinct seeded queries (a batch holds no query twice while batch <= queries)")
    ap.add_argument("--alg-queries", type=int, default=16,
                    help="queries whose stage sets are captured for the algorithmic bytes of the roofline")
    ap.add_argument("--serve-rate", type=float, default=600.0,
                    help="offered rate of the served phase of the bench line (Poisson arrivals)")
    ap.add_argument("--serve-phase-seconds", type=float, default=3.0)
    ap.add_argument("--autotune", metavar="CACHE", default=os.path.join(tempfile.gettempdir(), "msc_tune_c2.txt"),
                    help="tune the set kernels' launch shapes on the first 16 queries before timing (msc_autotune), "
                         "writing the choice to CACHE ('none': keep the default shapes)")
    ap.add_argument("--cpu-procs", type=int, default=16, help="processes of the all-core oracle leg")
    ap.add_argument("--cpu-queries", type=int, default=16, help="queries of the all-core oracle leg")
    ap.add_argument("--plain-steps", type=int, default=100)
    ap.add_argument("--cpu-replan", action="store_true",
                    help="replan workload: also time the oracle on query 0 (about two minutes)")
    ap.add_argument("--workspace-gb", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cone", type=int, nargs=3, metavar=("AZ_CDEG", "EL_CDEG", "HALF_CDEG"),
                    help="approach cone of the last segment for every query (a variant workload)")
    ap.add_argument("--plain-only", action="store_true",
                    help="stop after the plain phase (the run profiled for profiles/expand_trace_c2.md)")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_JSON"),
                    help="write profiles/expand_trace_c2.md from a kernel trace of a --plain-only run")
    ap.add_argument("--traffic-run", action="store_true",
                    help="run the program of the HBM counter passes (see profiles/expand_traffic_c2.md)")
    ap.add_argument("--traffic-out", default="gpurun_out/traffic_alg.json")
    ap.add_argument("--gms-summary", nargs=2, metavar=("KERNEL_STATS_CSV", "BENCH_JSON"),
                    help="write profiles/gap_search_2deg.md from a kernel-statistics run of --workload gms")
    ap.add_argument("--traffic-summary", nargs="+", metavar="CSV_OR_JSON",
                    help="FETCH_CSV WRITE_CSV ALG_JSON [TCC_CSV]: write profiles/expand_traffic_c2.md from the "
                         "counter passes (the optional third pass: TCC_HIT_sum and TCC_MISS_sum)")
    args = ap.parse_args()
    if args.gms_summary:
        return gms_summary(args)
    if args.traffic_summary:
        return traffic_summary(args)
    if args.trace_summary:
        return trace_summary(args)
    if args.c4_stages_summary:
        return c4_stages_summary(args)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.traffic_run:
        return traffic_run(args)
    if args.c4_stages_run:
        return c4_stages_run(args)
    if args.workload == "c2serve":
        return bench_c2serve(args)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "refine":
        return bench_refine(args)
    if args.workload == "replan":
        return bench_replan(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload in ("guided", "posepath"):
        return bench_guided(args)
    if args.workload == "short":
        return bench_short(args)
    if args.workload == "gms":
        return bench_gms(args)

    import torch

    from paper_1906_10678_amd import msc, synth

    solver = msc.Solver(0, workspace_bytes=args.workspace_gb << 30)
    cone = tuple(args.cone) if args.cone else None
    print("preparing %d queries" % args.queries, file=sys.stderr, flush=True)
    gen = synth.query_gms if args.arm == "gms" else synth.query_c2
    queries = []
    for s in range(args.queries):
        queries.append(gen(s, solver.pose_fn_for))
        if (s + 1) % 16 == 0:
            print("prepared %d queries" % (s + 1), file=sys.stderr, flush=True)
    arm = queries[0].arm
    n, na = queries[0].scene.n, arm.na

    # Algorithmic bytes per expansion launch, from one captured run of each of the first
    # 16 queries (the roofline sums the launches of those queries).
    alg, splits = [], []
    for i, q in enumerate(queries):
        scene = solver.scene(q.scene)
        if i >= args.alg_queries:
            solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta, approach=cone)
            splits.append(solver.stats()["split_m"])
            alg.append(None)
            continue
        st, _ = solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta, flags=msc.CAPTURE_SETS,
                            approach=cone)
        stats = solver.stats()
        splits.append(stats["split_m"])
        alg.append(expansion_bytes(solver, msc, n, na, stats))
        if (i + 1) % 4 == 0:
            print("captured %d queries" % (i + 1), file=sys.stderr, flush=True)
    print("captured stage sets; splits", splits, file=sys.stderr, flush=True)
    tuned = None
    if args.autotune and args.autotune != "none":
        specs = []
        for q in queries[:16]:
            specs.append(msc.QuerySpec(solver.scene(q.scene), q.arm, q.target, start=q.start, waypoints=q.waypoints,
                                       delta=q.max_delta))
        ts = time.perf_counter()
        entries = solver.autotune(specs, args.autotune, approach=cone)
        tuned = {"entries": len(entries), "non_default": sum(1 for e in entries if e[2] != 0),
                 "seconds": round(time.perf_counter() - ts, 2), "cache": args.autotune}
        print("autotune", tuned, entries, file=sys.stderr, flush=True)

    # ---- plain: one query per call, every launch timed with HIP events --------------
    # A query answered NO_REACH / NO_PATH is a complete solve (every retry was run);
    # only negative statuses are errors.
    statuses = {}
    def plain_step(i):
        q = queries[i % len(queries)]
        scene = solver.scene(q.scene)
        st, path = solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta, flags=msc.PROFILE,
                               approach=cone)
        if st < 0:
            raise RuntimeError("query %d: error status %d" % (i % len(queries), st))
        statuses[i % len(queries)] = st
        return solver.timings()

    for i in range(len(queries)):
        plain_step(i)
    torch.cuda.synchronize()
    lat, launches = [], []
    t0 = time.perf_counter()
    for i in range(args.plain_steps):
        ts = time.perf_counter()
        recs = plain_step(i)
        lat.append(time.perf_counter() - ts)
        launches.append((i % len(queries), recs))
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t0
    per_kernel = {}
    for _, recs in launches:
        for kname, stage, nin, nout, ms in recs:
            t = per_kernel.setdefault(kname, [0.0, 0])
            t[0] += ms
            t[1] += 1
    b_sum, ms_sum, cnt, transitions = 0.0, 0.0, 0, 0
    for qi, recs in launches:
        if alg[qi] is None:
            continue
        q = queries[qi]
        # the joint windows of the query's reach search: start +- W * delta, within the limits
        wlo = np.maximum(q.arm.lo_steps(), np.asarray(q.start) - q.waypoints * q.max_delta)
        whi = np.minimum(q.arm.hi_steps(), np.asarray(q.start) + q.waypoints * q.max_delta)
        for kname, stage, nin, nout, ms in recs:
            if kname in ("expand_fwd", "expand_bwd"):
                b_sum += alg[qi][(kname, stage)]
                ms_sum += ms
                cnt += 1
                j = stage - 1 if kname == "expand_fwd" else stage   # the joint the stage turns
                transitions += nin * int(whi[j] - wlo[j] + 1)
    achieved = b_sum / (ms_sum * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(),
                "l2_hit_rate": measured_traffic("L2 hit rate of the expansions"),
                "kernel": "expand (k_expand_fwd + k_expand_bwd)", "launches": cnt,
                "avg_launch_us": round(1e3 * ms_sum / max(cnt, 1), 2),
                "alg_bytes_per_launch": round(b_sum / max(cnt, 1)),
                "alg_bytes_max_launch": int(max(v for a in alg if a is not None for v in a.values())),
                "transitions_per_s": round(transitions / (ms_sum * 1e-3), 1),
                "transitions_per_launch": round(transitions / max(cnt, 1)),
                "alg_queries": sum(1 for a in alg if a is not None)}
    plain_lat = np.array(lat) * 1e3
    plain = {"solves_per_s": round(args.plain_steps / plain_wall, 3),
             "p50_ms": round(float(np.percentile(plain_lat, 50)), 4),
             "p99_ms": round(float(np.percentile(plain_lat, 99)), 4),
             "kernel_ms_per_query": {k: round(v[0] / args.plain_steps, 4) for k, v in sorted(per_kernel.items())}}
    print("plain", plain["solves_per_s"], "solves/s", file=sys.stderr, flush=True)
    if args.plain_only:
        # the run profiled for the kernel-trace summary: the plain phase is its last GPU work
        print(json.dumps({"plain": plain, "roofline": roofline, "queries": len(queries), "splits": splits}),
              flush=True)
        return

    # achievable HBM bandwidth on this device: a 1 GiB device-to-device copy (read + write)
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roofline["copy_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 5)
    # the kernels on full-size plans, where the sets stream from HBM (counter summary)
    roofline["large_stages"] = full_size_stages()

    # ---- batched: each step rasterises the scenes of a batch and solves it with msc_batch
    def batch_step(b):
        specs = []
        scenes = {}
        for j in range(args.batch):
            q = queries[(b * args.batch + j) % len(queries)]
            key = q.seed
            if key not in scenes:
                scenes[key] = solver.scene(q.scene)
            specs.append(msc.QuerySpec(scenes[key], q.arm, q.target, start=q.start, waypoints=q.waypoints,
                                       delta=q.max_delta))
        res = solver.batch(specs, approach=cone)
        for j, (st, _, _) in enumerate(res):
            qi = (b * args.batch + j) % len(queries)
            if st != statuses[qi]:
                raise RuntimeError("batched query %d: status %d, alone %d" % (qi, st, statuses[qi]))
        return [r[2] for r in res]

    lanes = args.lanes
    sweep = {}
    if lanes <= 0:
        for L in (2, 4, 8, 12, 16):
            solver.set_lanes(L)
            batch_step(0)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            batch_step(1)
            torch.cuda.synchronize()
            sweep[L] = args.batch / (time.perf_counter() - ts)
        lanes = max(sweep, key=sweep.get)
        print("lane sweep", {k: round(v, 1) for k, v in sweep.items()}, "->", lanes, file=sys.stderr, flush=True)
    solver.set_lanes(lanes)
    for b in range(args.warmup):
        batch_step(b)
    torch.cuda.synchronize()
    qlat = []
    t0 = time.perf_counter()
    for b in range(args.steps):
        qlat.extend(batch_step(b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    qlat = np.array(qlat)

    # ---- served: the same queries as a Poisson stream through the server, one lane (one
    # query at a time, the plain form) against the batch's lane count
    served = {"offered_per_s": args.serve_rate, "seconds": args.serve_phase_seconds,
              "p_latency": "per query, from submission to completion"}
    scenes = [solver.scene(q.scene) for q in queries]
    rng = np.random.default_rng(11)
    for key, L in (("one_lane", 1), ("lanes_%d" % lanes, lanes)):
        solver.set_lanes(L)
        solver.server_start(approach=cone)
        try:
            served[key] = serve_poisson(solver, msc, queries, scenes, args.serve_rate, args.serve_phase_seconds,
                                        rng)
        finally:
            solver.server_stop()
        print("served", key, served[key], file=sys.stderr, flush=True)
    solver.set_lanes(0)

    result = {
        "metric": "8-DOF reach+path solves/sec" + (" (4 segments x 2 DOF)" if args.arm == "gms" else ""),
        "value": round(args.steps * args.batch / wall, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "p50_ms": round(float(np.percentile(qlat, 50)), 4),
        "p99_ms": round(float(np.percentile(qlat, 99)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "8-DOF reach pose + 16-waypoint path queries: alternating yaw/pitch chain "
                               "30,30,25,25,20,20,15,10 voxels, +-170 deg in 5 deg steps, 256^3 bit-packed grid, "
                               "dilation 2, 32 boxes + 8 spheres, max 5 deg per joint per waypoint; a step is one "
                               "batch (scenes rasterised in the step) solved with msc_batch over worker lanes",
                   "batch": args.batch, "lanes": lanes, "lane_sweep": {str(k): round(v, 1) for k, v in sweep.items()},
                   "queries": len(queries), "grid": n, "dof": arm.dof, "waypoints": queries[0].waypoints,
                   "splits": splits, "statuses": [statuses[i] for i in range(len(queries))],
                   "approach_cone_cdeg": list(cone) if cone else None,
                   "arm": ("two DOF per segment: (yaw, length 0) + (pitch, length L), L = 60, 50, 40, 25 voxels"
                           if args.arm == "gms" else "alternating yaw/pitch chain"),
                   "p_latency": "per query, from batch start to its completion",
                   "autotune": tuned},
        "plain": plain,
        "served": served,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(queries, splits, cone, args.cpu_procs, args.cpu_queries)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
