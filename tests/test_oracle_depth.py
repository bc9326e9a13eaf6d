"""Pins of the oracle's depth buffer (Section 3.1, paragraph "Hybrid
Rendering": the distance at which a pixel's ray enters the first voxel whose
density is above a threshold, found by tracing the whole ray): an all-voxel
slab brute force on tiny grids, with and without the compositing's early stop
(which must not change the depth), and the hand-derived two-voxel column."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _slab(o, d, lo, hi):
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a]:
                return 1.0, 0.0
            continue
        u = (lo[a] - o[a]) / d[a]
        v = (hi[a] - o[a]) / d[a]
        t0 = max(t0, min(u, v))
        t1 = min(t1, max(u, v))
    return t0, t1


@pytest.mark.parametrize("lam", [0.0, 0.01, 0.5])
@pytest.mark.parametrize("depth,frac", [(1, 0.4), (2, 0.15), (3, 0.03)])
def test_depth_equals_brute_force(oracle_mod, depth, frac, lam):
    rng = np.random.default_rng(70 + depth)
    G = 1 << (depth + 1)
    occ = rng.random((G, G, G)) < frac
    cz, cy, cx = np.nonzero(occ.transpose(2, 1, 0))
    cells = np.stack([cx, cy, cz], axis=1)
    lin = (cells[:, 2] * G + cells[:, 1]) * G + cells[:, 0]
    order = np.argsort(lin)
    lin, cells = lin[order], cells[order]
    n = len(lin)
    sig = rng.uniform(0.0, 10.0, n)
    th = 5.0
    o = rng.uniform(-2.5, 2.5, (300, 3))
    d = rng.uniform(-0.9, 0.9, (300, 3)) - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = oracle_mod.render(o, d, depth, lin, np.arange(n), sig, np.zeros((n, 1)), lam, depth_sigma=th)
    h = 1.0 / (1 << depth)
    checked = found = 0
    for r in range(len(o)):
        if out["min_gap"][r] < 1e-9 * h:
            continue
        ta, tb = _slab(o[r], d[r], -np.ones(3), np.ones(3))
        ta = max(ta, 0.0)
        best = np.inf
        if tb > ta:
            for c, s in zip(cells, sig):
                if s <= th:
                    continue
                lo = -1.0 + c * h
                t0, t1 = _slab(o[r], d[r], lo, lo + h)
                t0, t1 = max(t0, ta), min(t1, tb)
                if t1 > t0:
                    best = min(best, t0)
        if np.isinf(best):
            assert np.isinf(out["dist"][r])
        else:
            found += 1
            assert abs(out["dist"][r] - best) < 1e-12
        checked += 1
    assert checked > 250 and found > 30
    if lam == 0.5:
        # on some rays the early stop ends the compositing before the depth
        # voxel is reached (its entry lies at or after the last composited exit)
        late = np.isfinite(out["dist"]) & (out["dist"] >= out["seg"][:, 3])
        assert late.sum() >= 1


def test_depth_golden_column(oracle_mod):
    with open(os.path.join(GOLDEN, "two_voxel_column.json")) as fh:
        g = json.load(fh)
    depth = g["depth"]
    G = 1 << (depth + 1)
    c = np.array(g["cells"])
    lin = (c[:, 2] * G + c[:, 1]) * G + c[:, 0]
    sig = np.array(g["sigma_over_ln2"]) * math.log(2.0)
    f = np.array(g["feat"])
    for case in g["depth_cases"]:
        out = oracle_mod.render(np.array([g["ray_origin"]]), np.array([g["ray_dir"]]), depth, lin,
                                np.array(g["leaf_ids"]), sig, f, case["lambda_th"], depth_sigma=case["threshold"])
        want = math.inf if case["depth"] == "inf" else case["depth"]
        assert out["dist"][0] == want, case
