"""Oracle of the short-reach shortcut and the path that follows it ("Short Reaches").

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the GPU library or its
binding.  It shares no code with the GPU path; it builds on the oracle's pinned staged
search (its forward sets), tables and pose replay, and on the waypoint walk of
``oracle.guided``.  Plain numpy; joint values are integer steps.

The paper adds a criterion to the reach search: as each segment hypothesis is tested
for collision along its length, it is also tested for a near encounter with the target;
a hypothesis that comes near the target with no collision before that point is a target
hit, and the hit with the shortest path becomes the path the arm follows (the segments
before it plus the sublength up to the hit, and a short bridge to the target).  In this
discrete model:

* A hypothesis of segment k (k = 2..K; segment 1 is the column the first joint only
  spins) is a state of the forward set F_{k-1} and an angle of joint k.  Its hit point is
  its first sample s (1..S) within squared distance ``rho2`` of the target, when samples
  1..s are all free and inside the grid.
* Its path length, in 1/S voxel, is S * (L_1 + ... + L_{k-1}) + s * L_k.  The shortcut is
  the hit of the least (length, squared distance of the hit point, k), and among the
  joint tuples (q_1..q_k) that realise such a hit the first in the canonical order of the
  reach search (reference 0: per joint |a| then a, joint 1 first).
* The pruned forward sets lose no hit when rho + 1 <= R_{k+1} (the next segment's
  reach radius) for every k <= K, which the caller must ensure (a hit lies within
  R_k + rho + 1 of its segment's start; the set keeps states within R_k + R_{k+1} + ...).
* The path: the end effector walks the shortcut back from the target: the hit point,
  the earlier samples of segment k, the samples of segments k-1..2, the end of segment 1
  (``oracle.guided`` walk, tracked joint = the end effector, from each reach pose in
  turn).  Without a hit, the reach-pose-guided path of ``oracle.guided`` is taken.

Parity status: pinned in tests/test_oracle_shortcut.py against a brute-force enumeration
of every valid joint prefix (no pruning, no marking, no walk), against a plain
recomputation of the hit point of the returned tuple, and by invariants of the path.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import NO_PATH, NO_REACH, OK, reach, reach_radii, tables
from . import guided


def _decode(keys: np.ndarray, N: int):
    keys = np.asarray(keys, np.uint64)
    ie = (keys & np.uint64(0xff)).astype(np.int64)
    ia = ((keys >> np.uint64(8)) & np.uint64(0xff)).astype(np.int64)
    v = (keys >> np.uint64(16)).astype(np.int64)
    return v % N, (v // N) % N, v // (N * N), ia, ie


def _key(N: int, x, y, z, ia, ie) -> np.ndarray:
    v = (np.asarray(z, np.int64) * N + np.asarray(y, np.int64)) * N + np.asarray(x, np.int64)
    return (v.astype(np.uint64) << np.uint64(16)) | (np.asarray(ia, np.uint64) << np.uint64(8)) | \
        np.asarray(ie, np.uint64)


def _turn(arm, k: int, ia, ie, a, na: int):
    if arm.types[k] == 0:
        return (ia + a) % na, ie
    return ia, (ie + a) % na


def _hit_of(occ, sweep, x, y, z, ia2, ie2, target, rho2):
    """For hypotheses starting at (x, y, z) along orientation (ia2, ie2): (sample index s
    1-based or 0 when no hit, squared distance of that sample)."""
    N = occ.shape[0]
    S = sweep.shape[2]
    pts = np.stack([x, y, z], axis=-1)[:, None, :] + sweep[ia2, ie2].astype(np.int64)   # (m, S, 3)
    inside = ((pts >= 0) & (pts < N)).all(axis=-1)
    cl = np.clip(pts, 0, N - 1)
    free = inside & (occ[cl[..., 2], cl[..., 1], cl[..., 0]] == 0)
    clear_upto = np.cumprod(free, axis=1).astype(bool)
    d2 = ((pts - np.asarray(target, np.int64)) ** 2).sum(axis=-1)
    hit = clear_upto & (d2 <= rho2)
    anyhit = hit.any(axis=1)
    s = np.where(anyhit, hit.argmax(axis=1) + 1, 0)
    sd2 = np.where(anyhit, d2[np.arange(len(s)), np.maximum(s - 1, 0)], 0)
    return s, sd2


def check_radius(arm, rho2: int, K: int) -> bool:
    """The pruned forward sets keep every hit: rho + 1 <= R_{k+1} for k = 2..K."""
    R = reach_radii(arm)
    rho = int(np.ceil(np.sqrt(rho2)))
    return 2 <= K <= len(arm.types) - 1 and all(rho + 1 <= R[k] for k in range(2, K + 1))


def shortcut(arm, occ, target, rho2: int, K: int, sets: dict):
    """The shortcut over the forward sets F_0..F_{K-1} of a reach search (keys of
    ``oracle.reach``): None, or dict(k, q[k], s, d2, length, point)."""
    N = occ.shape[0]
    na, S = 36000 // arm.step_cdeg, arm.samples
    lo, hi = guided.arm_lo(arm), guided.arm_hi(arm)
    target = np.asarray(target, np.int64)
    best = None                      # (length, d2, k)
    per_k = {}
    for k in range(2, K + 1):        # segment k, joint index k-1
        keys = sets[("F", k - 1)]
        if keys is None or len(keys) == 0:
            continue
        x, y, z, ia, ie = _decode(keys, N)
        _, sweep = tables(na, S, arm.lens[k - 1])
        base_len = S * int(sum(arm.lens[:k - 1]))
        rows = []
        for a in range(lo[k - 1], hi[k - 1] + 1):
            ia2, ie2 = _turn(arm, k - 1, ia, ie, a, na)
            s, d2 = _hit_of(occ, sweep, x, y, z, ia2, ie2, target, rho2)
            ok = s > 0
            if not ok.any():
                continue
            length = base_len + s * arm.lens[k - 1]
            rows.append((a, ok, s, d2, length))
            for i in np.flatnonzero(ok):
                key = (int(length[i]), int(d2[i]), k)
                if best is None or key < best:
                    best = key
        per_k[k] = (keys, rows)
    if best is None:
        return None
    length, bd2, k = best
    # D_{k-1}: states with an angle that realises the best hit
    keys, rows = per_k[k]
    win = np.zeros(len(keys), bool)
    for a, ok, s, d2, ln in rows:
        win |= ok & (ln == length) & (d2 == bd2)
    D = {k - 1: np.sort(keys[win])}
    for j in range(k - 1, 0, -1):    # D_{j-1} from D_j through joint j
        prev = sets[("F", j - 1)]
        x, y, z, ia, ie = _decode(prev, N)
        off, sweep = tables(na, S, arm.lens[j - 1])
        keep = np.zeros(len(prev), bool)
        for a in range(lo[j - 1], hi[j - 1] + 1):
            ia2, ie2 = _turn(arm, j - 1, ia, ie, a, na)
            d = off[ia2, ie2].astype(np.int64)
            nk = _key(N, x + d[:, 0], y + d[:, 1], z + d[:, 2], ia2, ie2)
            inD = np.isin(nk, D[j])
            if not inD.any():
                continue
            cl = _segment_clear(occ, sweep, x, y, z, ia2, ie2)
            keep |= inD & cl
        D[j - 1] = np.sort(prev[keep])
    # the canonical walk from the root
    x0, y0, z0, ia0, ie0 = [int(v[0]) for v in _decode(sets[("F", 0)][:1], N)]
    q = []
    cur = (x0, y0, z0, ia0, ie0)
    order = lambda j: sorted(range(lo[j], hi[j] + 1), key=lambda a: (abs(a), a))
    for j in range(1, k):
        off, sweep = tables(na, S, arm.lens[j - 1])
        x, y, z, ia, ie = cur
        for a in order(j - 1):
            ia2, ie2 = _turn(arm, j - 1, ia, ie, a, na)
            d = off[ia2, ie2]
            nxt = (x + int(d[0]), y + int(d[1]), z + int(d[2]), int(ia2), int(ie2))
            if not np.isin(_key(N, *nxt), D[j]).any():
                continue
            if not _segment_clear(occ, sweep, np.array([x]), np.array([y]), np.array([z]),
                                  np.array([ia2]), np.array([ie2]))[0]:
                continue
            q.append(a)
            cur = nxt
            break
        else:
            raise AssertionError("the walk found no move into D")
    _, sweep = tables(na, S, arm.lens[k - 1])
    x, y, z, ia, ie = cur
    for a in order(k - 1):
        ia2, ie2 = _turn(arm, k - 1, ia, ie, a, na)
        s, d2 = _hit_of(occ, sweep, np.array([x]), np.array([y]), np.array([z]), np.array([ia2]),
                        np.array([ie2]), target, rho2)
        if s[0] > 0 and S * int(sum(arm.lens[:k - 1])) + int(s[0]) * arm.lens[k - 1] == length and d2[0] == bd2:
            q.append(a)
            point = np.array([x, y, z]) + sweep[ia2, ie2, s[0] - 1].astype(np.int64)
            return {"k": k, "q": np.array(q, np.int64), "s": int(s[0]), "d2": int(d2[0]), "length": length,
                    "point": point}
    raise AssertionError("no move realises the best hit")


def _segment_clear(occ, sweep, x, y, z, ia2, ie2):
    N = occ.shape[0]
    pts = np.stack([x, y, z], axis=-1)[:, None, :] + sweep[ia2, ie2].astype(np.int64)
    inside = ((pts >= 0) & (pts < N)).all(axis=-1)
    cl = np.clip(pts, 0, N - 1)
    return (inside & (occ[cl[..., 2], cl[..., 1], cl[..., 0]] == 0)).all(axis=1)


def shortcut_waypoints(arm, hit) -> np.ndarray:
    """The end effector's walk back from the target along the shortcut: the hit point and
    the earlier samples of segment k, the samples of segments k-1..2 (end to start; none
    for length 0), then the end of segment 1."""
    k, s = hit["k"], hit["s"]
    pts = guided.sample_points(guided.sub_arm(arm, k), hit["q"])
    walk = [pts[k - 1][i] for i in range(s - 1, -1, -1)]
    for j in range(k - 2, 0, -1):
        if arm.lens[j] == 0:
            continue
        walk.extend(pts[j][i] for i in range(arm.samples - 1, -1, -1))
    walk.append(pts[0][arm.samples - 1])
    return np.array(walk, np.int64)


def short_path(arm, occ, target, rho2: int = 4, K: Optional[int] = None, tracked: Optional[int] = None,
               delta: int = 1, delta2: int = 2, eps2: int = 9, retries: int = 4):
    """(status, rows root pose first .. reach pose, hit or None, reach result).  With a hit
    the end effector follows the shortcut from each reach pose in turn; without one the
    reach-pose-guided path (``tracked``, default n - 2) is taken."""
    n = len(arm.types)
    K = min(4, n - 1) if K is None else K
    r = reach(arm, occ, target, m=max(K - 1, 1), want=retries, keep_sets=True)
    if r.status != OK:
        return r.status, None, None, r
    hit = shortcut(arm, occ, target, rho2, K, r.sets)
    if hit is not None:
        pts, trk = shortcut_waypoints(arm, hit), n
    else:
        trk = n - 2 if tracked is None else tracked
    for i in range(min(retries, len(r.sols))):
        qs = np.asarray(r.sols[i], np.int64)
        if hit is None:
            pts = guided.reach_waypoints(arm, qs, trk)
        rows, _ = guided.track(arm, occ, qs, pts, trk, delta, delta2, eps2)
        if rows is not None:
            r.index = i
            return OK, rows[::-1].astype(np.int32), hit, r
    return NO_PATH, None, hit, r
