"""Pins of the oracle's ray indexing and compositing (Eq. 5-6): brute-force
all-voxel slab tests on tiny grids, closed forms, invariants and a hand-derived
worked example (CPU)."""
import json
import math
import os

import numpy as np
import pytest

import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lin(c, G):
    return (c[..., 2] * G + c[..., 1]) * G + c[..., 0]


def _random_occupancy(rng, depth, frac):
    G = 1 << (depth + 1)
    occ = rng.random((G, G, G)) < frac
    cz, cy, cx = np.nonzero(occ.transpose(2, 1, 0))
    c = np.stack([cx, cy, cz], axis=1)
    lin = _lin(c, G)
    order = np.argsort(lin)
    return lin[order], np.arange(len(lin))[order] * 3 + 1, c[order]


def _random_rays(rng, n):
    o = rng.uniform(-2.5, 2.5, (n, 3))
    # half the rays aim at random points inside the root, some are axis-aligned
    tgt = rng.uniform(-0.95, 0.95, (n, 3))
    d = tgt - o
    k = n // 8
    d[:k] = 0.0
    ax = rng.integers(0, 3, k)
    d[np.arange(k), ax] = rng.choice([-1.0, 1.0], k)
    o[np.arange(k), ax] = np.where(d[np.arange(k), ax] > 0, -1.7, 1.7)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


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


def _brute_force_hits(o, d, depth, cells, leaves):
    """All-voxel slab test: every occupied cell with a positive-length overlap
    with the clipped ray, ordered by entry."""
    h = 1.0 / (1 << depth)
    ta, tb = _slab(o, d, -np.ones(3), np.ones(3))
    ta = max(ta, 0.0)
    if not tb > ta:
        return [], []
    rows = []
    for c, leaf in zip(cells, leaves):
        lo = -1.0 + c * h
        t0, t1 = _slab(o, d, lo, lo + h)
        t0, t1 = max(t0, ta), min(t1, tb)
        if t1 > t0:
            rows.append((t0, int(leaf), t1 - t0))
    rows.sort()
    return [r[1] for r in rows], [r[2] for r in rows]


@pytest.mark.parametrize("depth,frac", [(1, 0.5), (2, 0.3), (3, 0.15)])
def test_partition_equals_brute_force(oracle_mod, depth, frac):
    rng = np.random.default_rng(10 + depth)
    lin, leaf, cells = _random_occupancy(rng, depth, frac)
    N = int(leaf.max()) + 1
    o, d = _random_rays(rng, 600)
    out = oracle_mod.render(o, d, depth, lin, leaf, np.ones(N), np.zeros((N, 1)), 0.0,
                            max_hits=3 * (1 << (depth + 1)) + 4)
    h = 1.0 / (1 << depth)
    checked = 0
    for r in range(len(o)):
        if out["min_gap"][r] < 1e-9 * h:
            continue
        bl, bd = _brute_force_hits(o[r], d[r], depth, cells, leaf)
        n = int(out["n_comp"][r])
        assert n == len(bl) == out["n_hit"][r]
        assert list(out["hit_leaf"][r, :n]) == bl
        assert np.allclose(out["hit_delta"][r, :n], bd, rtol=0, atol=1e-12)
        checked += 1
    assert checked > 500


def test_segment_lengths_cover_clip(oracle_mod):
    # with every cell occupied the samples tile the clipped ray exactly
    depth = 2
    G = 1 << (depth + 1)
    c = np.stack(np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij"), -1).reshape(-1, 3)
    lin = np.sort(_lin(c, G))
    leaf = np.arange(len(lin))
    rng = np.random.default_rng(3)
    o, d = _random_rays(rng, 400)
    out = oracle_mod.render(o, d, depth, lin, leaf, np.zeros(len(lin)), np.zeros((len(lin), 1)),
                            0.0, max_hits=3 * G + 4)
    for r in range(len(o)):
        ta, tb = _slab(o[r], d[r], -np.ones(3), np.ones(3))
        ta = max(ta, 0.0)
        total = out["hit_delta"][r, :out["n_comp"][r]].sum()
        expect = max(tb - ta, 0.0)
        assert abs(total - expect) < 1e-12


def test_axis_aligned_row_has_leaf_chords(oracle_mod):
    depth = 3
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    c = np.array([[x, 5, 9] for x in range(G)])
    lin = _lin(c, G)
    leaf = np.arange(G)
    o = np.array([[-1.5, -1.0 + 5.3 * h, -1.0 + 9.7 * h]])
    d = np.array([[1.0, 0.0, 0.0]])
    out = oracle_mod.render(o, d, depth, lin, leaf, np.zeros(G), np.zeros((G, 1)), 0.0,
                            max_hits=G)
    assert out["n_comp"][0] == G
    assert list(out["hit_leaf"][0]) == list(range(G))
    assert np.all(out["hit_delta"][0] == h)


def test_single_voxel_closed_form(oracle_mod):
    depth = 2
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    cell = np.array([[3, 4, 2]])
    lin = _lin(cell, G)
    rng = np.random.default_rng(7)
    lo = -1.0 + cell[0] * h
    sig = np.array([17.0])
    f = np.array([[0.3, -1.2, 2.0]])
    for _ in range(200):
        o = rng.uniform(-3, 3, 3)
        d = (lo + rng.uniform(0.05, 0.95, 3) * h) - o
        d /= np.linalg.norm(d)
        t0, t1 = _slab(o, d, lo, lo + h)
        ell = t1 - max(t0, 0.0)
        out = oracle_mod.render(o[None], d[None], depth, lin, np.array([0]), sig, f, 0.0)
        A = 1.0 - math.exp(-sig[0] * ell)
        assert abs(out["A"][0] - A) < 1e-14
        assert abs(out["T"][0] - math.exp(-sig[0] * ell)) < 1e-14
        assert np.allclose(out["F"][0], A * f[0], atol=1e-14)


def _tiny_render(oracle_mod, lam, pose=True):
    s = sg.make_scene("tiny")
    r, R, T = sg.make_poses(s.J, 1)
    if not pose:
        r = np.zeros_like(r)
    B = oracle_mod.fk(s.parent, s.rest_joint, r, R, T)[0]
    ok, ol, _, _, _ = oracle_mod.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B)
    K, c2w = sg.make_cameras(s, 1, 64, 64)
    o, d = oracle_mod.camera_rays(K, c2w, 64, 64)
    return s, oracle_mod.render(o.reshape(-1, 3), d.reshape(-1, 3), s.depth, ok, ol, s.sigma,
                                s.feat, lam, max_hits=400)


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_weights_plus_transmittance_is_one(oracle_mod, lam):
    _, out = _tiny_render(oracle_mod, lam)
    assert np.all(np.abs(out["A"] + out["T"] - 1.0) < 1e-13)
    assert (out["n_hit"] > 0).mean() > 0.1


def test_early_stop_rule(oracle_mod):
    s, full = _tiny_render(oracle_mod, 0.0)
    _, stop = _tiny_render(oracle_mod, 0.01)
    stopped = 0
    for r in range(len(full["A"])):
        n = int(full["n_comp"][r])
        T = 1.0
        expect = n
        for i in range(n):
            T *= math.exp(-float(s.sigma[full["hit_leaf"][r, i]]) * full["hit_delta"][r, i])
            if T < 0.01:
                expect = i + 1
                break
        assert stop["n_comp"][r] == expect
        stopped += expect < n
        assert np.array_equal(stop["hit_leaf"][r, :expect], full["hit_leaf"][r, :expect])
    assert stopped > 100
    # after the stop the remaining transmittance is below lambda_th (opacity above 1 - lambda_th)
    cut = stop["n_comp"] < full["n_comp"]
    assert np.all(stop["T"][cut] < 0.01)


def test_axis_column_closed_form(oracle_mod):
    depth = 3
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    rng = np.random.default_rng(11)
    xs = np.array([2, 3, 4, 7, 8, 12])
    c = np.array([[x, 6, 6] for x in xs])
    lin = _lin(c, G)
    sig = rng.uniform(1.0, 9.0, len(xs))
    f = rng.normal(size=(len(xs), 4))
    o = np.array([[-1.2, -1.0 + 6.5 * h, -1.0 + 6.25 * h]])
    d = np.array([[1.0, 0.0, 0.0]])
    out = oracle_mod.render(o, d, depth, lin, np.arange(len(xs)), sig, f, 0.0)
    T = 1.0
    F = np.zeros(4)
    for i in range(len(xs)):
        F += math.exp(-h * sig[:i].sum()) * (1.0 - math.exp(-sig[i] * h)) * f[i]
    assert np.allclose(out["F"][0], F, atol=1e-14)
    assert abs(out["T"][0] - math.exp(-h * sig.sum())) < 1e-15


def test_infinite_density_returns_first_feature(oracle_mod):
    depth = 2
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    c = np.array([[x, 1, 1] for x in range(2, 6)])
    lin = _lin(c, G)
    f = np.arange(12.0).reshape(4, 3)
    for sig0 in (np.inf, 1e6):
        sig = np.array([sig0, 3.0, 3.0, 3.0])
        o = np.array([[-1.5, -1.0 + 1.5 * h, -1.0 + 1.5 * h]])
        out = oracle_mod.render(o, np.array([[1.0, 0.0, 0.0]]), depth, lin, np.arange(4), sig, f, 0.0)
        assert np.allclose(out["F"][0], f[0], atol=1e-12)
        assert out["T"][0] < 1e-12


def test_golden_two_voxel_column(oracle_mod):
    with open(os.path.join(GOLDEN, "two_voxel_column.json")) as fh:
        g = json.load(fh)
    depth = g["depth"]
    G = 1 << (depth + 1)
    lin = _lin(np.array(g["cells"]), G)
    sig = np.array(g["sigma_over_ln2"]) * math.log(2.0)
    f = np.array(g["feat"])
    for case in g["cases"]:
        out = oracle_mod.render(np.array([g["ray_origin"]]), np.array([g["ray_dir"]]), depth, lin,
                                np.array(g["leaf_ids"]), sig, f, case["lambda_th"])
        assert np.allclose(out["F"][0], case["F"], atol=1e-15)
        assert abs(out["A"][0] - case["A"]) < 1e-15
        assert abs(out["T"][0] - case["T"]) < 1e-15
        assert out["n_comp"][0] == case["n_comp"]


def test_identity_pose_render_equals_canonical(oracle_mod):
    s = sg.make_scene("tiny")
    B = oracle_mod.fk(s.parent, s.rest_joint, np.zeros((1, s.J, 3)), np.zeros((1, 3)),
                      np.zeros((1, 3)))[0]
    ok, ol, _, _, _ = oracle_mod.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B)
    ck, cl = oracle_mod.canonical_occupancy(s.ijk, s.depth)
    K, c2w = sg.make_cameras(s, 1, 48, 48)
    o, d = oracle_mod.camera_rays(K, c2w, 48, 48)
    a = oracle_mod.render(o.reshape(-1, 3), d.reshape(-1, 3), s.depth, ok, ol, s.sigma, s.feat, 0.01)
    b = oracle_mod.render(o.reshape(-1, 3), d.reshape(-1, 3), s.depth, ck, cl, s.sigma, s.feat, 0.01)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["A"], b["A"])


def test_rays_unit_and_through_pixel_centres(oracle_mod):
    s = sg.make_scene("tiny")
    K, c2w = sg.make_cameras(s, 2, 20, 30)
    o, d = oracle_mod.camera_rays(K, c2w, 20, 30)
    assert np.allclose(np.linalg.norm(d, axis=-1), 1.0, atol=1e-15)
    # project back: pixel (x, y) centre lands at (x + 1/2, y + 1/2)
    for v in range(2):
        Rm = c2w[v, :, :3]
        dc = d[v] @ Rm
        u = K[v, 0, 0] * dc[..., 0] / dc[..., 2] + K[v, 0, 2]
        w = K[v, 1, 1] * dc[..., 1] / dc[..., 2] + K[v, 1, 2]
        xs, ys = np.meshgrid(np.arange(30) + 0.5, np.arange(20) + 0.5)
        assert np.allclose(u, xs, atol=1e-10) and np.allclose(w, ys, atol=1e-10)


def test_bf16_rounding(oracle_mod):
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 1e-40, 65504.0], dtype=np.float32)
    y = oracle_mod.bf16_round(x)
    # exactly representable stays; halfway rounds to even; generic rounds to nearest
    assert y[0] == 1.0 and y[1] == 1.0 and y[2] == 1.0078125
    assert abs(float(y[3]) + 3.140625) < 1e-12
    assert np.all((y.view(np.uint32) & 0xFFFF) == 0)
    normal = np.abs(x) >= np.finfo(np.float32).tiny
    assert np.all(np.abs(y - x)[normal] <= np.abs(x)[normal] * 2.0 ** -8)
    # against the library's float32 -> bfloat16 conversion (round to nearest even)
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    z = (rng.normal(size=20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(z).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(oracle_mod.bf16_round(z), ref)
