"""GPU parity at the full-size workload (1.5M leaves, 40 bones, C = 16, 8
cameras at 512x512), in the launch configuration bench.py times: all 8 views
of a pose rendered by one compositing launch.  The oracle computes sampled
pixels one by one; the posed octree is compared whole."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, guard_leaves, log, make_renderer

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
POSES = [0, 29]   # first and last pose of the benchmark batch


@pytest.fixture(scope="module")
def full():
    s = sg.make_scene("full")
    cfg = sg.CONFIGS["full"]
    r_, R_, T_ = sg.make_poses(s.J, 30, cfg.pose_seed0)
    sel = (r_[POSES], R_[POSES], T_[POSES])
    K, c2w = sg.make_cameras(s, cfg.n_views, cfg.height, cfg.width)
    rend = make_renderer(s, sel, K, c2w, cfg.height, cfg.width)
    B = oracle.fk(s.parent, s.rest_joint, *sel)
    return s, rend, B, K, c2w, cfg


@pytest.mark.parametrize("pi", [0, 1], ids=["pose0", "pose29"])
def test_full_octree_bit_exact(full, pi):
    """Posed keys, occupied cells, winners and the brick level of a pose against
    the oracle's set constructions.  A leaf whose posed centre lies within
    1e-9 h of a lattice plane (the rounding guard band) may land in either
    cell; the cells such a leaf can reach (its key on either side) are left
    out of the comparison, everything else is compared exactly, and the brick
    rows are checked for consistency with the GPU's own cell list."""
    s, rend, B, *_ = full
    log(f"full: posed keys + octree of pose {POSES[pi]}")
    pt = oracle.lbs(s.ijk, s.depth, s.bone, s.weight, B[pi])
    cells, valid = oracle.posed_cells(pt, s.depth)
    ko = oracle.posed_keys(cells, valid)
    kg = rend.get_posed_keys(pi)
    band = guard_leaves(pt, s.depth)
    log(f"  {int(band.sum())} leaves in the guard band")
    assert band.sum() <= 5
    assert np.array_equal(kg[~band], ko[~band])
    g = rend.get_octree(pi)
    o = oracle.posed_octree(ko)
    assert g["collisions"] > 0
    skip = set(int(k) for k in np.concatenate([kg[band], ko[band]]) if k != 0xFFFFFFFF)
    gw = {int(k): int(w) for k, w in zip(g["keys"], g["winner"]) if int(k) not in skip}
    ow = {int(k): int(w) for k, w in zip(o["keys"], o["winner"]) if int(k) not in skip}
    assert gw == ow
    skip_b = set(k >> 9 for k in skip)
    gb = {int(b): m for b, m in zip(g["brick_keys"], g["brick_mask"]) if int(b) not in skip_b}
    ob = {int(b): m for b, m in zip(o["brick_keys"], o["brick_mask"]) if int(b) not in skip_b}
    assert gb.keys() == ob.keys()
    assert all(np.array_equal(gb[b], ob[b]) for b in gb)
    if not skip:
        for k in ["keys", "winner", "brick_keys", "brick_row", "brick_mask"]:
            assert np.array_equal(g[k], o[k]), k
    # every brick row points at the first cell of its brick in the GPU's list
    keys, rows, bk = g["keys"].astype(np.int64), g["brick_row"], g["brick_keys"].astype(np.int64)
    assert np.all(keys[rows] >> 9 == bk)
    assert np.all(rows[1:] > rows[:-1]) and rows[0] == 0
    assert np.all(keys[rows[1:] - 1] >> 9 == bk[:-1])


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_full_sampled_pixels(full, lam):
    s, rend, B, K, c2w, cfg = full
    sig, f = flut(s)
    H, W = cfg.height, cfg.width
    log(f"full: render 2 poses x 8 views x {H}x{W}, lambda {lam}")
    F, A, T = rend.render(sig, f, lambda_th=lam)
    F = F.cpu().numpy()
    A = A.cpu().numpy()
    o, d = oracle.camera_rays(K, c2w, H, W)
    h = 1.0 / (1 << s.depth)
    rng = np.random.default_rng(11)
    for p in range(len(POSES)):
        ok_, ol_, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(K.shape[0]):
            hitpix = np.flatnonzero(A[p, v].reshape(-1) > 0)
            pix = np.concatenate([rng.choice(hitpix, 600, replace=False), rng.integers(0, H * W, 200)])
            ref = oracle.render(o[v].reshape(-1, 3)[pix], d[v].reshape(-1, 3)[pix], s.depth, ok_, ol_,
                                s.sigma, s.feat, lam)
            good = (ref["min_gap"] >= 1e-9 * h) & (ref["min_tgap"] >= 1e-5)
            assert good.mean() > 0.99
            Fg = F[p, v].reshape(s.C, -1)[:, pix][:, good]
            Fr = ref["F"][good].T
            rel = np.abs(Fg - Fr).max() / np.abs(Fr).max()
            arel = np.abs(A[p, v].reshape(-1)[pix][good] - ref["A"][good]).max() / ref["A"].max()
            log(f"  pose {POSES[p]} view {v}: F rel_max {rel:.2e}, A rel_max {arel:.2e}")
            assert rel <= TOL_F32 and arel <= TOL_F32


def test_full_hit_lists_sampled(full):
    s, rend, B, K, c2w, cfg = full
    sig, f = flut(s)
    H, W = cfg.height, cfg.width
    v = 3
    log("full: hit lists of pose 0 view 3 (lambda 0)")
    leaf, delta, cnt = rend.get_hits(0, v, sig, f, lambda_th=0.0, max_hits=320)
    o, d = oracle.camera_rays(K[v:v + 1], c2w[v:v + 1], H, W)
    ok_, ol_, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[0])
    rng = np.random.default_rng(5)
    pix = rng.choice(np.flatnonzero(cnt > 0), 1500, replace=False)
    ref = oracle.render(o.reshape(-1, 3)[pix], d.reshape(-1, 3)[pix], s.depth, ok_, ol_, s.sigma, s.feat,
                        0.0, max_hits=320)
    h = 1.0 / (1 << s.depth)
    good = ref["min_gap"] >= 1e-9 * h
    assert good.mean() > 0.99
    for j, i in enumerate(pix):
        if not good[j]:
            continue
        assert cnt[i] == ref["n_comp"][j]
        c = min(int(cnt[i]), 320)
        assert np.array_equal(leaf[i, :c], ref["hit_leaf"][j, :c])
        assert np.allclose(delta[i, :c], ref["hit_delta"][j, :c], rtol=1e-12, atol=1e-12)
