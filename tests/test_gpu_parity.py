"""GPU parity of the plain renderer against the FP64 oracle, through the C ABI.

Indices (posed keys, winners, bricks, hit lists) must be bit-exact; feature and
opacity maps within 1e-5 rel_max (FP32 compositing, FP64 geometry).  Rays or
leaves inside the rounding guard band (a partition gap below 1e-9 h, a centre
within 1e-9 h of a lattice plane, T within 1e-5 relative of lambda_th) are
excluded from the bit-exact / 1e-5 checks and counted."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, guard_leaves, log, make_renderer, map_error, oracle_maps

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def tiny():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    r_, R_, T_ = sg.make_poses(s.J, 3)
    # pose 0: identity; pose 1: random; pose 2: random with a global rotation/translation
    r_[0] = 0.0
    R_[2] = [0.2, -0.1, 0.3]
    T_[2] = [0.03, -0.02, 0.01]
    K, c2w = sg.make_cameras(s, 2, 128, 128)
    rend = make_renderer(s, (r_, R_, T_), K, c2w, 128, 128)
    B = oracle.fk(s.parent, s.rest_joint, r_, R_, T_)
    return s, rend, B, K, c2w, (r_, R_, T_)


def test_fk_matches_oracle(tiny):
    s, rend, B, *_ = tiny
    log("fk: tiny scene, 3 poses")
    Bg = rend.get_bones()
    assert np.allclose(Bg, B, rtol=0, atol=1e-14)


def test_posed_keys_bit_exact(tiny):
    s, rend, B, *_ = tiny
    for p in range(B.shape[0]):
        log(f"posed keys: pose {p}")
        kg = rend.get_posed_keys(p)
        pt = oracle.lbs(s.ijk, s.depth, s.bone, s.weight, B[p])
        cells, valid = oracle.posed_cells(pt, s.depth)
        ko = oracle.posed_keys(cells, valid)
        band = guard_leaves(pt, s.depth)
        assert band.sum() <= 2
        assert np.array_equal(kg[~band], ko[~band])


def test_identity_pose_keys_shift(tiny):
    s, rend, B, *_ = tiny
    kg = rend.get_posed_keys(0)
    c = s.ijk.T.astype(np.int64) + (1 << (s.depth - 1))
    assert np.array_equal(kg, oracle.morton30(c).astype(np.uint32))


def test_octree_bit_exact(tiny):
    s, rend, B, *_ = tiny
    for p in range(B.shape[0]):
        log(f"octree: pose {p}")
        g = rend.get_octree(p)
        pt = oracle.lbs(s.ijk, s.depth, s.bone, s.weight, B[p])
        cells, valid = oracle.posed_cells(pt, s.depth)
        o = oracle.posed_octree(oracle.posed_keys(cells, valid))
        assert np.array_equal(g["keys"], o["keys"])
        assert np.array_equal(g["winner"], o["winner"])
        assert np.array_equal(g["brick_keys"], o["brick_keys"])
        assert np.array_equal(g["brick_row"], o["brick_row"])
        assert np.array_equal(g["brick_mask"], o["brick_mask"])
        assert g["dropped"] == o["dropped"]
        assert g["collisions"] == s.n - o["dropped"] - len(o["keys"])


def test_hit_lists_bit_exact(tiny):
    s, rend, B, K, c2w, _ = tiny
    sig, f = flut(s)
    h = 1.0 / (1 << s.depth)
    for p in range(B.shape[0]):
        for v in range(K.shape[0]):
            log(f"hit lists: pose {p} view {v} (lambda 0)")
            leaf, delta, cnt = rend.get_hits(p, v, sig, f, lambda_th=0.0, max_hits=200)
            ref = oracle_maps(s, B[p:p + 1], K[v:v + 1], c2w[v:v + 1], 128, 128, 0.0, max_hits=200)[0][0]
            ok = ref["min_gap"] >= 1e-9 * h
            assert (~ok).sum() <= 4
            assert np.array_equal(cnt[ok], ref["n_comp"][ok])
            n = 0
            for i in np.nonzero(ok & (cnt > 0))[0]:
                c = min(int(cnt[i]), 200)
                assert np.array_equal(leaf[i, :c], ref["hit_leaf"][i, :c]), f"ray {i}"
                assert np.allclose(delta[i, :c], ref["hit_delta"][i, :c], rtol=1e-12, atol=1e-12)
                n += 1
            assert n > 1000


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_feature_maps_match_oracle(tiny, lam):
    s, rend, B, K, c2w, _ = tiny
    sig, f = flut(s)
    log(f"render: tiny, 3 poses x 2 views, lambda {lam}")
    F, A, T = rend.render(sig, f, lambda_th=lam)
    F = F.cpu().numpy()
    A = A.cpu().numpy()
    T = T.cpu().numpy()
    ref = oracle_maps(s, B, K, c2w, 128, 128, lam)
    h = 1.0 / (1 << s.depth)
    for p in range(B.shape[0]):
        for v in range(K.shape[0]):
            r = ref[p][v]
            ok = (r["min_gap"] >= 1e-9 * h) & (r["min_tgap"] >= 1e-5)
            assert (~ok).mean() < 0.01
            Fr = r["F"].T.reshape(s.C, 128 * 128)
            Fg = F[p, v].reshape(s.C, -1)
            emax, emean = map_error(Fg, Fr, ok)
            amax, _ = map_error(A[p, v].reshape(-1), r["A"], ok)
            log(f"  pose {p} view {v}: F rel_max {emax:.2e} rel_mean {emean:.2e}, A rel_max {amax:.2e}")
            assert emax <= TOL_F32 and amax <= TOL_F32
            assert np.allclose(T[p, v].reshape(-1)[ok], r["T"][ok], rtol=0, atol=1e-5)
            # empty pixels are exactly zero / transmittance one
            miss = r["n_hit"] == 0
            assert np.all(Fg[:, miss] == 0) and np.all(A[p, v].reshape(-1)[miss] == 0)
            assert np.all(T[p, v].reshape(-1)[miss] == 1)


def test_identity_pose_equals_canonical_render(tiny):
    s, rend, B, K, c2w, _ = tiny
    sig, f = flut(s)
    F, A, _ = rend.render(sig, f, lambda_th=0.01)
    F = F.cpu().numpy()
    ck, cl = oracle.canonical_occupancy(s.ijk, s.depth)
    o, d = oracle.camera_rays(K, c2w, 128, 128)
    for v in range(K.shape[0]):
        r = oracle.render(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, ck, cl, s.sigma, s.feat, 0.01)
        ok = r["min_tgap"] >= 1e-5
        emax, _ = map_error(F[0, v].reshape(s.C, -1), r["F"].T, ok)
        assert emax <= TOL_F32


def test_forward_is_deterministic(tiny):
    s, rend, *_ = tiny
    sig, f = flut(s)
    a = rend.render(sig, f)
    b = rend.render(sig, f)
    for x, y in zip(a, b):
        assert bool((x == y).all())
    st = rend.stats()
    assert st["rays"] == 3 * 2 * 128 * 128 and st["samples"] > 0


@pytest.mark.parametrize("bf16", [False, True], ids=["f32", "bf16"])
def test_background_in_kernel_equals_background_kernel(tiny, monkeypatch, bf16):
    """The compositing kernel's waves write the background pixels (tiles with
    no brick) of the forward maps and the depth buffer; the separate
    background kernel (ARTEMIS_BG_KERNEL=1) must give the same maps bit for
    bit, and both count every ray."""
    s, rend, *_ = tiny
    sig, f = flut(s, "bf16" if bf16 else "f32")
    th = float(np.median(s.sigma))
    a = rend.render(sig, f, 0.01, fp32_geom=bf16)
    da = rend.render_depth(sig, f, th, 0.01, fp32_geom=bf16)
    st_a = rend.stats()
    monkeypatch.setenv("ARTEMIS_BG_KERNEL", "1")
    b = rend.render(sig, f, 0.01, fp32_geom=bf16)
    db = rend.render_depth(sig, f, th, 0.01, fp32_geom=bf16)
    st_b = rend.stats()
    for x, y in zip(a + da, b + db):
        assert bool((x == y).all())
    assert st_a["rays"] == st_b["rays"] == 3 * 2 * 128 * 128
    # background pixels exist in these maps, and they hold F = 0, A = 0, T = 1
    F, A, T = a
    bgpix = T == 1.0
    assert int(bgpix.sum()) > 0 and bool((A[bgpix] == 0).all())
