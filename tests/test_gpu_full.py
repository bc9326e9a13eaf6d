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


def test_full_octree_bit_exact(full):
    s, rend, B, *_ = full
    log("full: posed keys + octree of pose 0")
    pt = oracle.lbs(s.ijk, s.depth, s.bone, s.weight, B[0])
    cells, valid = oracle.posed_cells(pt, s.depth)
    ko = oracle.posed_keys(cells, valid)
    kg = rend.get_posed_keys(0)
    band = guard_leaves(pt, s.depth)
    assert band.sum() <= 5
    assert np.array_equal(kg[~band], ko[~band])
    if band.sum() == 0:
        g = rend.get_octree(0)
        o = oracle.posed_octree(ko)
        for k in ["keys", "winner", "brick_keys", "brick_row", "brick_mask"]:
            assert np.array_equal(g[k], o[k]), k
        assert g["collisions"] > 0


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
