"""The launch-shape autotuner (msc_autotune, msc_tune_load) through the C ABI: results
after tuning equal those before (and the oracle's on small queries), the choice survives
a round trip through its cache file, and foreign or malformed files are refused."""
import numpy as np
import pytest

import oracle
from paper_1906_10678_amd import msc, synth

from cases import tiny_case
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def _specs(solver):
    specs, ref = [], []
    for seed in range(4):
        q = synth.query_c2(seed, solver.pose_fn_for)
        sc = solver.scene(q.scene)
        specs.append(msc.QuerySpec(sc, q.arm, q.target, start=q.start, waypoints=q.waypoints, delta=q.max_delta))
        ref.append(None)
    for seed in range(6):
        arm, scene, rng = tiny_case(seed, dof=4)
        occ = oracle.raster(scene)
        qs = synth.candidate_poses(rng, arm, 300)
        ok, ends = oracle.poses(arm, occ, qs)
        t = ends[np.flatnonzero(ok)[0]]
        specs.append(msc.QuerySpec(solver.scene(scene), arm, t))
        r = oracle.reach(arm, occ, t, keep_sets=False)
        ref.append((r.status, r.pose))
    return specs, ref


def test_autotune_keeps_results_and_round_trips(solver, tmp_path):
    specs, ref = _specs(solver)
    before = [(st, None if v is None else v.copy()) for st, v, _ in solver.batch(specs)]
    for (st, v), r in zip(before, ref):
        if r is not None:
            assert st == r[0] and (st != msc.OK or np.array_equal(v, r[1]))
    cache = str(tmp_path / "tune.txt")
    say("autotune", len(specs), "queries")
    entries = solver.autotune(specs, cache)
    assert entries, "nothing tuned"
    kinds = {e[0] for e in entries}
    assert kinds <= {"expand_fwd", "expand_bwd", "join", "dmark"}
    after = solver.batch(specs)
    for (st, v), (st2, v2, _) in zip(before, after):
        assert st == st2 and (st != msc.OK or np.array_equal(v, v2))
    # round trip: clear by loading a file with no entries, then the cache back
    text = open(cache).read().splitlines()
    assert text[0] == "msc-tune 1" and text[1].startswith("device ")
    empty = tmp_path / "empty.txt"
    empty.write_text("\n".join(text[:2]) + "\n")
    solver.tune_load(str(empty))
    assert solver.tune_entries() == []
    solver.tune_load(cache)
    assert solver.tune_entries() == entries


def test_tune_load_refuses_other_files(solver, tmp_path):
    before = solver.tune_entries()
    bad = tmp_path / "bad.txt"
    bad.write_text("hello\n")
    with pytest.raises(msc.MscError) as e:
        solver.tune_load(str(bad))
    assert e.value.status == msc.E_ARG
    other = tmp_path / "other.txt"
    other.write_text("msc-tune 1\ndevice gfx000\n")
    with pytest.raises(msc.MscError) as e:
        solver.tune_load(str(other))
    assert e.value.status == msc.E_STATE
    dev = tmp_path / "dev.txt"
    good_dev = None
    import ctypes
    # the device line of a real cache (the tuner writes it)
    specs, _ = _specs(solver)
    path = str(tmp_path / "real.txt")
    solver.autotune(specs[-2:], path)
    good_dev = open(path).read().splitlines()[1]
    dev.write_text("msc-tune 1\n%s\nentry 5 3 99 16384 0\n" % good_dev)
    with pytest.raises(msc.MscError) as e:
        solver.tune_load(str(dev))
    assert e.value.status == msc.E_ARG
    dev.write_text("msc-tune 1\n%s\nentry 5 3 1 999 0\n" % good_dev)
    with pytest.raises(msc.MscError) as e:
        solver.tune_load(str(dev))
    assert e.value.status == msc.E_ARG
    # refused files leave the choice as it was
    solver.tune_load(path)
    kept = solver.tune_entries()
    with pytest.raises(msc.MscError):
        solver.tune_load(str(bad))
    assert solver.tune_entries() == kept
