"""Edge cases of the HIP path against the FP64 oracle: ragged images, other
channel counts, shallow octrees, empty and degenerate views, cameras inside the
posed root and inside the object, axis-aligned rays, every leaf dropped,
several pose batches, tile-list overflow re-runs and ABI error paths."""
import math
import os

import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, log, make_renderer, map_error

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _compare(scene, rend, B, K, c2w, H, W, lam, F=None, A=None, T=None, sigma=None, feat=None):
    import torch
    if F is None:
        sig = torch.from_numpy(scene.sigma if sigma is None else sigma).cuda()
        f = torch.from_numpy(scene.feat if feat is None else feat).cuda()
        F, A, T = rend.render(sig, f, lambda_th=lam)
    F = F.cpu().numpy()
    A = A.cpu().numpy()
    T = T.cpu().numpy()
    o, d = oracle.camera_rays(K, c2w, H, W)
    h = 1.0 / (1 << scene.depth)
    worst = 0.0
    for p in range(B.shape[0]):
        ok_, ol_, _, _, _ = oracle.pose_occupancy(scene.ijk, scene.depth, scene.bone, scene.weight, B[p])
        for v in range(K.shape[0]):
            r = oracle.render(o[v].reshape(-1, 3), d[v].reshape(-1, 3), scene.depth, ok_, ol_,
                              scene.sigma if sigma is None else sigma, scene.feat if feat is None else feat,
                              lam)
            good = (r["min_gap"] >= 1e-9 * h) & (r["min_tgap"] >= 1e-5)
            assert good.mean() > 0.98
            Fr = r["F"].T
            Fg = F[p, v].reshape(Fr.shape[0], -1)
            if np.abs(Fr[:, good]).max() > 0:
                emax, _ = map_error(Fg, Fr, good)
                worst = max(worst, emax)
                assert emax <= TOL_F32
            else:
                assert np.all(Fg[:, good] == 0)
            assert np.allclose(A[p, v].reshape(-1)[good], r["A"][good], rtol=0, atol=1e-5)
            assert np.allclose(T[p, v].reshape(-1)[good], r["T"][good], rtol=0, atol=1e-5)
    return worst


@pytest.mark.parametrize("H,W", [(37, 53), (1, 1), (8, 64), (129, 7)])
def test_ragged_images(H, W):
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 2)
    K, c2w = sg.make_cameras(s, 3, H, W)
    log(f"ragged image {H}x{W}")
    rend = make_renderer(s, poses, K, c2w, H, W)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    _compare(s, rend, B, K, c2w, H, W, 0.01)


@pytest.mark.parametrize("C", [4, 32])
def test_other_channel_counts(C):
    s = sg.make_scene("tiny", C=C)
    poses = sg.make_poses(s.J, 1)
    K, c2w = sg.make_cameras(s, 2, 64, 64)
    log(f"C = {C}")
    rend = make_renderer(s, poses, K, c2w, 64, 64)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    _compare(s, rend, B, K, c2w, 64, 64, 0.0)


def _random_octree(depth, n, J, seed):
    """A random sparse canonical octree with a short bone chain."""
    rng = np.random.default_rng(seed)
    G = 1 << depth
    cells = rng.choice(G ** 3, size=n, replace=False)
    ijk = np.stack([cells % G, (cells // G) % G, cells // (G * G)]).astype(np.uint16)
    parent = np.arange(-1, J - 1, dtype=np.int32)
    rest = np.zeros((J, 3))
    rest[1:, 0] = np.linspace(0.1, 0.3, J - 1)
    bone = np.stack([rng.permutation(J)[:4] if J >= 4 else rng.integers(0, J, 4) for _ in range(n)]).T
    w = rng.random((4, n))
    w /= w.sum(axis=0, keepdims=True)
    scene = sg.Scene(sg.CONFIGS["tiny"], depth, ijk, bone.astype(np.uint8), w.astype(np.float32),
                     parent, rest, rng.uniform(1, 40, n).astype(np.float32),
                     rng.normal(size=(n, 8)).astype(np.float32), 1.0, np.zeros(3), 0.8)
    return scene


@pytest.mark.parametrize("depth,n", [(1, 5), (2, 30), (3, 300)])
def test_shallow_octrees(depth, n):
    s = _random_octree(depth, n, 5, 100 + depth)
    poses = sg.make_poses(s.J, 2, max_deg=20.0)
    K, c2w = sg.make_cameras(s, 3, 48, 40)
    log(f"shallow octree depth {depth}, {n} leaves")
    rend = make_renderer(s, poses, K, c2w, 48, 40)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    _compare(s, rend, B, K, c2w, 48, 40, 0.0)
    # hit lists of the first view, bit-exact
    import torch
    sig, f = torch.from_numpy(s.sigma).cuda(), torch.from_numpy(s.feat).cuda()
    leaf, delta, cnt = rend.get_hits(0, 0, sig, f, lambda_th=0.0, max_hits=64)
    o, d = oracle.camera_rays(K[:1], c2w[:1], 48, 40)
    ok_, ol_, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[0])
    r = oracle.render(o.reshape(-1, 3), d.reshape(-1, 3), s.depth, ok_, ol_, s.sigma, s.feat, 0.0, max_hits=64)
    good = r["min_gap"] >= 1e-9 / (1 << depth)
    assert np.array_equal(cnt[good], r["n_comp"][good])
    for i in np.flatnonzero(good & (cnt > 0)):
        assert np.array_equal(leaf[i, :cnt[i]], r["hit_leaf"][i, :cnt[i]])


def test_single_leaf_and_camera_inside_object():
    s = _random_octree(4, 1, 1, 7)
    s.sigma[:] = 10.0
    poses = (np.zeros((1, 1, 3)), np.zeros((1, 3)), np.zeros((1, 3)))
    c = -0.5 + (s.ijk[:, 0].astype(float) + 0.5) / 16
    # camera centre inside the only leaf, looking along an arbitrary direction
    K = np.array([[[20.0, 0, 8], [0, 20.0, 8], [0, 0, 1]]])
    Rm = sg.rotation_about(np.array([0.3, -0.5, 0.8]), 0.7)
    c2w = np.concatenate([Rm, (c + 0.01)[:, None]], axis=1)[None]
    log("camera inside the single leaf")
    rend = make_renderer(s, poses, K, c2w, 16, 16)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    _compare(s, rend, B, K, c2w, 16, 16, 0.0)


def test_camera_looking_away_and_inside_root():
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 1)
    K, c2w = sg.make_cameras(s, 2, 32, 32)
    c2w = c2w.copy()
    c2w[0, :, :3] = c2w[0, :, :3] @ np.diag([-1.0, 1.0, -1.0])   # turned around: every ray misses
    c2w[1, :, 3] = [0.7, 0.7, 0.3]                                 # inside the posed root
    rend = make_renderer(s, poses, K, c2w, 32, 32)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    import torch
    F, A, T = rend.render(*flut(s), lambda_th=0.01)
    assert bool((F[0, 0] == 0).all()) and bool((A[0, 0] == 0).all()) and bool((T[0, 0] == 1).all())
    _compare(s, rend, B, K, c2w, 32, 32, 0.01, F, A, T)


def test_axis_aligned_rays():
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 1)
    # camera looking along -z from above, principal point on a pixel centre:
    # the centre ray is exactly axis-parallel
    K = np.array([[[30.0, 0, 16.5], [0, 30.0, 16.5], [0, 0, 1]]])
    Rm = np.array([[1.0, 0, 0], [0, -1.0, 0], [0, 0, -1.0]])
    c2w = np.concatenate([Rm, np.array([[0.013], [0.021], [1.6]])], axis=1)[None]
    log("axis-aligned rays")
    rend = make_renderer(s, poses, K, c2w, 33, 33)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    _compare(s, rend, B, K, c2w, 33, 33, 0.0)


def test_all_leaves_dropped():
    s = sg.make_scene("tiny")
    r_, R_, T_ = sg.make_poses(s.J, 1)
    T_[0] = [5.0, 0.0, 0.0]
    K, c2w = sg.make_cameras(s, 1, 32, 32)
    rend = make_renderer(s, (r_, R_, T_), K, c2w, 32, 32)
    F, A, T = rend.render(*flut(s), lambda_th=0.01)
    assert bool((A == 0).all()) and bool((T == 1).all()) and bool((F == 0).all())
    st = rend.stats()
    assert st["dropped"] == s.n and st["samples"] == 0


def test_pose_batches_and_overflow_reruns(monkeypatch):
    """A tiny slot budget splits the poses into several batches and a tiny
    initial tile-list capacity forces the overflow re-run, for the forward
    and the adjoint; both must give the same results as the default path."""
    import torch
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 5)
    K, c2w = sg.make_cameras(s, 3, 64, 64)
    sig, f = flut(s)
    rng = np.random.default_rng(2)
    dF = torch.from_numpy(rng.normal(size=(5, 3, s.C, 64, 64)).astype(np.float32)).cuda()
    ref = make_renderer(s, poses, K, c2w, 64, 64)
    F0, A0, T0 = ref.render(sig, f, lambda_th=0.01)
    ds0, df0 = ref.backward(sig, f, F0, T0, dF, None, lambda_th=0.01)
    monkeypatch.setenv("ARTEMIS_SLOT_BUDGET_MB", "1")
    monkeypatch.setenv("ARTEMIS_PAIR_CAP", "64")
    log("forced pose batches + tile-list overflow")
    alt = make_renderer(s, poses, K, c2w, 64, 64)
    F1, A1, T1 = alt.render(sig, f, lambda_th=0.01)
    assert bool((F1 == F0).all()) and bool((A1 == A0).all()) and bool((T1 == T0).all())
    ds1, df1 = alt.backward(sig, f, F1, T1, dF, None, lambda_th=0.01)
    assert torch.allclose(ds1, ds0, rtol=1e-5, atol=1e-6 * float(ds0.abs().max()))
    assert torch.allclose(df1, df0, rtol=1e-5, atol=1e-6 * float(df0.abs().max()))
    assert alt.stats()["launches"] > ref.stats()["launches"]


def test_abi_error_paths():
    import torch
    import paper_2202_05628_amd as art
    from paper_2202_05628_amd import ArtemisError, _lib

    s = sg.make_scene("tiny")
    r = art.Renderer(0)
    sig, f = flut(s)
    rc = r.lib.art_render(r._h, 8, 0, art._tptr(sig), art._tptr(f), 0.01, 0, art._tptr(sig),
                          art._tptr(sig), None)
    assert rc == _lib.ART_ESTATE                    # nothing loaded yet
    with pytest.raises(ArtemisError) as e:
        r.load_octree(6, np.concatenate([s.ijk[:, :10], s.ijk[:, :1]], axis=1))
    assert e.value.status == _lib.ART_EINVAL        # duplicate cell
    with pytest.raises(ArtemisError) as e:
        r.load_octree(6, np.full((3, 4), 64, dtype=np.uint16))
    assert e.value.status == _lib.ART_EINVAL        # outside the grid
    r.set_scene(s)
    bad = s.bone.copy()
    bad[0, 0] = 200
    r.set_skin(bad, s.weight)
    r.set_poses(*sg.make_poses(s.J, 1))
    K, c2w = sg.make_cameras(s, 1, 16, 16)
    r.set_cameras(K, c2w, 16, 16)
    with pytest.raises(ArtemisError) as e:
        r.render(sig, f)
    assert e.value.status == _lib.ART_EINVAL        # bone id >= J
    r.set_skin(s.bone, s.weight)
    with pytest.raises(ArtemisError) as e:
        r.render(sig, f, lambda_th=1.5)
    assert e.value.status == _lib.ART_EINVAL
    f6 = torch.zeros((s.n, 6), device="cuda")
    with pytest.raises(ArtemisError) as e:
        r.render(sig, f6)
    assert e.value.status == _lib.ART_EUNSUPPORTED
    c2 = c2w.copy()
    c2[0, :, 0] *= 2.0
    with pytest.raises(ArtemisError) as e:
        r.set_cameras(K, c2, 16, 16)
    assert e.value.status == _lib.ART_EINVAL        # not orthonormal
    # the context still works after the failures
    F, A, T = r.render(sig, f)
    assert float(A.max()) > 0
