"""The full-size 8-DOF reach + 16-waypoint path workload (seeds 0..15, the queries the
benchmark cycles over) against stored oracle answers, through the C ABI."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1906_10678_amd import msc, synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_c2_paths import fingerprint  # noqa: E402

with open(os.path.join(HERE, "golden", "c2_paths.json")) as f:
    GOLDEN = json.load(f)["queries"]


@pytest.mark.gpu
@pytest.mark.parametrize("row", GOLDEN, ids=lambda r: "seed%d" % r["seed"])
def test_c2_path_matches_oracle(solver, row):
    print("c2 golden seed", row["seed"], flush=True)
    q = synth.query_c2(row["seed"], solver.pose_fn_for)
    assert fingerprint(q) == row["fingerprint"], "stored answers are stale: rerun tests/golden/make_c2_paths.py"
    scene = solver.scene(q.scene)
    st, path = solver.path(scene, q.arm, q.start, q.target, q.waypoints, q.max_delta)
    assert st == row["status"]
    if st == msc.OK:
        assert np.array_equal(path, np.asarray(row["path"], np.int32))


def test_c2_golden_file_is_complete():
    assert [r["seed"] for r in GOLDEN] == list(range(16))
    for r in GOLDEN:
        assert r["status"] in (0, 1, 2)
        if r["status"] == 0:
            p = np.asarray(r["path"])
            assert p.shape == (17, 8)
            assert np.abs(np.diff(p, axis=0)).max() <= 1
            assert tuple(p[-1]) == tuple(r["reach_poses"][0]) or any(tuple(p[-1]) == tuple(x) for x in r["reach_poses"])
