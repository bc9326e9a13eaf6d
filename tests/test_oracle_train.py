"""Pins of the training-step oracle (oracle/train.py): the voxel regularisation
term of Eq. 10, the point-query operator Q and the projected Adam update."""
import numpy as np
import pytest

import oracle
import oracle.train as otr

INV = oracle.INVALID_KEY


def test_vrt_zero_without_collisions():
    rng = np.random.default_rng(1)
    keys = rng.permutation(1000)[:200].astype(np.int64)
    f = rng.normal(size=(200, 4))
    L, g, nv = otr.vrt(keys, f, 0.7)
    assert L == 0.0 and not g.any() and nv == 200


def test_vrt_two_voxel_collision_by_hand():
    # leaves 0 and 1 share cell 5 (leaf 0, the smaller id, wins), leaf 2 is
    # alone, leaf 3 left the posed root: N_v = 3.
    # L = lam / 3 * (|1 - 3| + |2 - (-1)|) = 5 lam / 3;
    # dL/df_0 = lam / 3 * sign(f_0 - f_1) = lam / 3 * (-1, +1), dL/df_1 = -dL/df_0.
    lam = 0.3
    keys = np.array([5, 5, 9, INV], dtype=np.int64)
    f = np.array([[1.0, 2.0], [3.0, -1.0], [0.0, 0.0], [7.0, 7.0]])
    L, g, nv = otr.vrt(keys, f, lam)
    assert nv == 3
    assert L == pytest.approx(5 * lam / 3, rel=1e-15)
    np.testing.assert_allclose(g[0], [-lam / 3, lam / 3], rtol=1e-15)
    np.testing.assert_allclose(g[1], [lam / 3, -lam / 3], rtol=1e-15)
    assert not g[2].any() and not g[3].any()


def test_vrt_matches_pairwise_brute_force():
    rng = np.random.default_rng(2)
    N, C = 300, 5
    keys = rng.integers(0, 40, N).astype(np.int64)
    keys[rng.random(N) < 0.1] = INV
    f = rng.normal(size=(N, C))
    lam = 1.3
    L, g, nv = otr.vrt(keys, f, lam)
    # winner of each leaf: the smallest index among all leaves with its key
    inside = [i for i in range(N) if keys[i] != INV]
    Lb = 0.0
    gb = np.zeros_like(f)
    for i in inside:
        w = min(j for j in range(N) if keys[j] == keys[i])
        Lb += np.abs(f[w] - f[i]).sum()
        gb[w] += np.sign(f[w] - f[i])
        gb[i] -= np.sign(f[w] - f[i])
    assert nv == len(inside)
    assert L == pytest.approx(lam * Lb / len(inside), rel=1e-13)
    np.testing.assert_allclose(g, lam * gb / len(inside), rtol=1e-13, atol=0)


def test_vrt_gradient_central_differences():
    rng = np.random.default_rng(3)
    N, C = 120, 3
    keys = rng.integers(0, 25, N).astype(np.int64)
    f = rng.normal(size=(N, C))
    lam = 0.9
    _, g, _ = otr.vrt(keys, f, lam)
    eps = 1e-6
    for _ in range(40):
        i, c = int(rng.integers(N)), int(rng.integers(C))
        fp, fm = f.copy(), f.copy()
        fp[i, c] += eps
        fm[i, c] -= eps
        fd = (otr.vrt(keys, fp, lam)[0] - otr.vrt(keys, fm, lam)[0]) / (2 * eps)
        assert fd == pytest.approx(g[i, c], abs=1e-8)


def test_query_matches_brute_force():
    rng = np.random.default_rng(4)
    depth = 3
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    N = 400
    cells = rng.integers(0, G, (N, 3))
    keys = oracle.morton30(cells).astype(np.int64)
    keys[rng.random(N) < 0.05] = INV
    # points: inside occupied cells, inside empty ones, and outside the root
    pts = np.concatenate([(cells[:200] + rng.random((200, 3))) * h - 1.0,
                          rng.uniform(-1.0, 1.0, (200, 3)),
                          rng.uniform(-2.0, 2.0, (100, 3))])
    got = otr.query(pts, depth, keys)
    for n, p in enumerate(pts):
        c = np.floor((p + 1.0) / h).astype(np.int64)
        hits = [i for i in range(N) if keys[i] != INV and np.array_equal(cells[i], c)]
        assert got[n] == (min(hits) if hits else -1)
    assert (got >= 0).sum() > 150


def test_flut_adam_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=(50, 4))
    grads = [rng.normal(size=(50, 4)) for _ in range(3)]
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k, gk in enumerate(grads):
        opt.zero_grad()
        t.grad = torch.tensor(gk)
        opt.step()
        with torch.no_grad():
            t.clamp_(min=0.0)
        p, m, v = otr.flut_adam(p, m, v, gk, k + 1, 0.05, lower=0.0)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-15)
