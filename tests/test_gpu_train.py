"""The FLUT training step through the C ABI: the voxel regularisation term
(Eq. 10) with its gradient, the point-query operator Q and the projected Adam
update against the FP64 oracle (oracle/train.py), then a training run that
fits a FLUT to seeded target maps.

The VRT decisions (which leaf wins a cell, the sign of f_w - f_i) are exact
on both sides: the posed keys are bit-exact outside the rounding guard band
(no leaf of these scenes lies within 1e-9 h of a cell face), and the sign of a
rounded FP32 difference is the sign of the exact one.  The gradient entries
are sums of +-lambda / N_v; the loss is summed in FP64."""
import numpy as np
import pytest

import oracle
import oracle.train as otr
import scenegen as sg
from gpu_common import guard_leaves, log, make_renderer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 3)
    K, c2w = sg.make_cameras(s, 2, 48, 40)
    rend = make_renderer(s, poses, K, c2w, 48, 40)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    keys = []
    for p in range(B.shape[0]):
        _, _, cells, valid, pt = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        assert not guard_leaves(pt[valid], s.depth).any()
        keys.append(oracle.posed_keys(cells, valid).astype(np.int64))
    return s, rend, B, keys, K, c2w


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_vrt_matches_oracle(tiny, storage):
    import torch
    s, rend, B, keys, _, _ = tiny
    f = torch.from_numpy(s.feat).cuda()
    if storage == "bf16":
        f = f.to(torch.bfloat16)
    f_np = f.float().cpu().numpy().astype(np.float64)
    lam = 0.25
    L, g = rend.vrt(f.contiguous(), lam)
    Lr, gr = 0.0, np.zeros_like(f_np)
    scales = []
    for p, k in enumerate(keys):
        lp, gp, nv = otr.vrt(k, f_np, lam)
        Lr += lp
        gr += gp
        scales.append(lam / nv)
    g = g.cpu().numpy().astype(np.float64)
    log(f"vrt {storage}: loss {L:.6f} vs oracle {Lr:.6f}; {int((gr != 0).any(axis=1).sum())} leaves with gradient")
    assert Lr > 0
    assert L == pytest.approx(Lr, rel=1e-6)
    np.testing.assert_allclose(g, gr, rtol=1e-5, atol=1e-6 * min(scales))


def test_vrt_accumulates_into_the_gradient(tiny):
    import torch
    s, rend, _, _, _, _ = tiny
    f = torch.from_numpy(s.feat).cuda()
    base = torch.full_like(f, 0.5)
    L1, g1 = rend.vrt(f, 0.25)
    L2, g2 = rend.vrt(f, 0.25, d_feat=base.clone())
    assert L1 == pytest.approx(L2, rel=1e-12)
    assert torch.allclose(g2 - 0.5, g1, atol=1e-6)
    L0, g0 = rend.vrt(f, 0.0)
    assert L0 == 0.0 and not g0.any()


def test_query_matches_oracle(tiny):
    import torch
    s, rend, B, keys, _, _ = tiny
    rng = np.random.default_rng(12)
    h = 1.0 / (1 << s.depth)
    for p in range(B.shape[0]):
        _, _, cells, valid, pt = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        pts = np.concatenate([pt[rng.choice(len(pt), 3000)],                      # posed leaf centres
                              (cells[rng.choice(len(pt), 2000)] + rng.random((2000, 3))) * h - 1.0,
                              rng.uniform(-1.0, 1.0, (2000, 3)),
                              rng.uniform(-1.5, 1.5, (500, 3))])
        got = rend.query(p, torch.from_numpy(pts).cuda()).cpu().numpy()
        want = otr.query(pts, s.depth, keys[p])
        log(f"query pose {p}: {int((want >= 0).sum())} of {len(pts)} points in occupied cells")
        assert np.array_equal(got, want)


def test_flut_adam_matches_oracle(tiny):
    import torch
    s, rend, _, _, _, _ = tiny
    rng = np.random.default_rng(13)
    n = 10007
    p0 = rng.normal(size=n).astype(np.float32)
    p = torch.from_numpy(p0).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    mabs = np.zeros(n)   # the first moment of |g|: scale of the FP32 rounding of m (m may cancel)
    # the hyper-parameters as the kernel receives them (FP32 values)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (0.05, 0.9, 0.999, 1e-8))
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32) * 10.0 ** rng.uniform(-3, 1, n).astype(np.float32)
        rend.flut_adam(p, torch.from_numpy(g).cuda(), m, v, step, lr, b1, b2, eps, lower=0.0)
        pr, mr, vr = otr.flut_adam(pr, mr, vr, g.astype(np.float64), step, lr, b1, b2, eps, lower=0.0)
        mabs = 0.9 * mabs + 0.1 * np.abs(g)
    np.testing.assert_allclose(p.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    assert np.all(np.abs(m.cpu().numpy() - mr) <= 1e-6 * mabs)
    np.testing.assert_allclose(v.cpu().numpy(), vr, rtol=1e-5, atol=0)
    assert (p.cpu().numpy() >= 0).all()


def test_training_step_gradient_matches_oracle(tiny):
    """The gradient a training step applies (adjoint of the map loss + VRT)
    against the oracle's: oracle.backward over every ray + oracle VRT."""
    import torch
    s, rend, B, keys, K, c2w = tiny
    H, W = rend.H, rend.W
    rng = np.random.default_rng(14)
    sig = torch.from_numpy(s.sigma).cuda()
    f = torch.from_numpy(s.feat).cuda()
    Ft = torch.from_numpy(rng.normal(size=(rend.P, rend.V, f.shape[1], H, W)).astype(np.float32)).cuda()
    F, A, T = rend.render(sig, f, 0.01)
    R = float(rend.P * rend.V * H * W)
    dF = (F - Ft) / R
    ds, df = rend.backward(sig, f, F, T, dF, None, 0.01)
    lam = 0.25
    _, df = rend.vrt(f, lam, d_feat=df)
    o, d = oracle.camera_rays(K, c2w, H, W)
    gs = np.zeros(s.n)
    gf = np.zeros((s.n, f.shape[1]))
    dF_np = dF.cpu().numpy().astype(np.float64)
    for p in range(B.shape[0]):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(rend.V):
            gF = dF_np[p, v].reshape(f.shape[1], -1).T
            a, b = oracle.backward(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, ok, ol, s.sigma, s.feat,
                                   0.01, gF)
            gs += a
            gf += b
        gf += otr.vrt(keys[p], s.feat.astype(np.float64), lam)[1]
    e_s = np.abs(ds.cpu().numpy() - gs).max() / np.abs(gs).max()
    e_f = np.abs(df.cpu().numpy() - gf).max() / np.abs(gf).max()
    log(f"training-step gradient: dsigma rel_max {e_s:.2e}, dfeat rel_max {e_f:.2e}")
    assert e_s <= 1e-4 and e_f <= 1e-4


def test_training_step_segmented_equals_unsegmented(tiny):
    """A training step with the segmented adjoint (checkpoints every 3
    samples) applies the unsegmented step's update: the same losses (the
    maps are the same bit for bit) and the same parameters up to the order of
    the gradient's float sums."""
    import torch
    s, rend, *_ = tiny
    rng = np.random.default_rng(16)
    Ft = torch.from_numpy(rng.normal(size=(rend.P, rend.V, s.C, rend.H, rend.W)).astype(np.float32)).cuda()
    out = {}
    for seg in ((4, 3), "off"):
        sig = torch.from_numpy(s.sigma).cuda()
        f = torch.from_numpy(s.feat).cuda()
        st = rend.train_state(sig, f)
        loss = rend.train_step(sig, f, st, Ft, lr=0.01, lambda_vrt=0.05, segments=seg)
        out[str(seg)] = (loss, sig.cpu().numpy(), f.cpu().numpy())
    (la, sa, fa), (lb, sb, fb) = out["(4, 3)"], out["off"]
    log(f"segmented training step: losses {la} / {lb}; max |d sigma| {np.abs(sa - sb).max():.2e}, "
        f"max |d f| {np.abs(fa - fb).max():.2e}")
    assert la["map"] == lb["map"]                       # the same maps
    assert abs(la["vrt"] - lb["vrt"]) <= 1e-9 * max(1.0, abs(lb["vrt"]))   # summed with atomics
    # Adam's first step moves a parameter by lr g / (|g| + eps): about lr sign(g)
    # where |g| >> eps, where a change of g's last bits changes nothing; where
    # |g| is near eps the step follows g's summation order
    s0, f0 = s.sigma.astype(np.float32), s.feat.astype(np.float32)
    big_s = np.abs(sb - s0) >= 0.005
    big_f = np.abs(fb - f0) >= 0.005
    assert big_s.mean() > 0.05 and big_f.mean() > 0.05
    # within 4 units in the last place of the value, or 1e-6 for values near 0
    close = lambda x, y: np.abs(x - y) <= np.maximum(4 * np.spacing(np.maximum(np.abs(x), np.abs(y))), 1e-6)
    assert close(sa, sb)[big_s].all() and close(fa, fb)[big_f].all()
    assert np.abs(sa - sb).max() <= 0.02 and np.abs(fa - fb).max() <= 0.02


def test_training_step_after_tile_list_overflow(tiny, monkeypatch):
    """With tile lists too small for the call, the step's asynchronous render
    reports the overflow and the step renders again (with its checkpoints)
    before the adjoint: the losses and the update equal those of a step
    without overflow."""
    import torch
    s, rend, _, _, K, c2w = tiny
    rng = np.random.default_rng(17)
    Ft = torch.from_numpy(rng.normal(size=(rend.P, rend.V, s.C, rend.H, rend.W)).astype(np.float32)).cuda()
    monkeypatch.setenv("ARTEMIS_PAIR_CAP", "64")   # every tile list overflows
    small = make_renderer(s, sg.make_poses(s.J, 3), K, c2w, 48, 40)
    seen = []
    status = small.render_status
    small.render_status = lambda: seen.append(status()) or seen[-1]   # record what the step read
    out = []
    for r in (small, rend):
        sig = torch.from_numpy(s.sigma).cuda()
        f = torch.from_numpy(s.feat).cuda()
        st = r.train_state(sig, f)
        loss = r.train_step(sig, f, st, Ft, lr=0.01, segments=(4, 3))
        out.append((loss, sig.cpu().numpy(), f.cpu().numpy()))
    monkeypatch.delenv("ARTEMIS_PAIR_CAP")
    small.close()
    assert seen and seen[0]["overflowed_items"] > 0   # the step's first render did overflow
    (la, sa, fa), (lb, sb, fb) = out
    log(f"training step after overflow: losses {la} / {lb}; max |d sigma| {np.abs(sa - sb).max():.2e}, "
        f"max |d f| {np.abs(fa - fb).max():.2e}")
    assert la["map"] == lb["map"]
    s0, f0 = s.sigma.astype(np.float32), s.feat.astype(np.float32)
    big_s, big_f = np.abs(sb - s0) >= 0.005, np.abs(fb - f0) >= 0.005
    assert big_s.mean() > 0.05 and big_f.mean() > 0.05
    close = lambda x, y: np.abs(x - y) <= np.maximum(4 * np.spacing(np.maximum(np.abs(x), np.abs(y))), 1e-6)
    assert close(sa, sb)[big_s].all() and close(fa, fb)[big_f].all()
    assert np.abs(sa - sb).max() <= 0.02 and np.abs(fa - fb).max() <= 0.02


def test_training_fits_target_maps(tiny):
    """Targets rendered from a seeded FLUT; training starts from another seeded
    FLUT.  The map loss falls by a large factor; with the VRT on, the features
    of colliding leaves end closer to their cell winner's than without it."""
    import torch
    s, rend, B, keys, _, _ = tiny
    rng = np.random.default_rng(15)
    sig_t = torch.from_numpy(s.sigma).cuda()
    f_t = torch.from_numpy(s.feat).cuda()
    Ft, At, _ = rend.render(sig_t, f_t, 0.01)
    results = {}
    for lam in (0.0, 0.05):
        sig = torch.from_numpy(rng.uniform(5, 50, s.n).astype(np.float32)).cuda()
        f = torch.from_numpy(rng.normal(size=s.feat.shape).astype(np.float32)).cuda()
        st = rend.train_state(sig, f)
        first = rend.train_step(sig, f, st, Ft, At, lr=0.05, lambda_vrt=lam)
        for _ in range(150):
            last = rend.train_step(sig, f, st, Ft, At, lr=0.05, lambda_vrt=lam)
        vrt_end, _ = rend.vrt(f, 1.0)
        results[lam] = (first["map"], last["map"], vrt_end)
        log(f"lambda_vrt {lam}: map loss {first['map']:.4f} -> {last['map']:.4f}, VRT measure {vrt_end:.4f}")
        assert (sig >= 0).all()
    for lam, (a, b, _) in results.items():
        assert b < 0.2 * a, lam
    assert results[0.05][2] < results[0.0][2]


def test_vrt_with_leaves_outside_the_root():
    """A global translation pushes part of the animal out of the posed root:
    the dropped leaves have no Q and N_v counts only the leaves inside."""
    import torch
    s = sg.make_scene("tiny")
    r, R, T = sg.make_poses(s.J, 2)
    T = T.copy()
    T[0] = [0.8, 0.0, 0.0]
    T[1] = [0.0, -0.7, 0.3]
    K, c2w = sg.make_cameras(s, 1, 16, 16)
    rend = make_renderer(s, (r, R, T), K, c2w, 16, 16)
    B = oracle.fk(s.parent, s.rest_joint, r, R, T)
    f = torch.from_numpy(s.feat).cuda()
    lam = 0.5
    L, g = rend.vrt(f, lam)
    Lr, gr, dropped = 0.0, np.zeros(s.feat.shape), 0
    for p in range(2):
        _, _, cells, valid, pt = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        assert not guard_leaves(pt[valid], s.depth).any()
        lp, gp, nv = otr.vrt(oracle.posed_keys(cells, valid).astype(np.int64), s.feat.astype(np.float64), lam)
        Lr += lp
        gr += gp
        dropped += s.n - nv
    log(f"vrt with {dropped} dropped leaf-poses: loss {L:.6f} vs {Lr:.6f}")
    assert dropped > 1000
    assert L == pytest.approx(Lr, rel=1e-6)
    np.testing.assert_allclose(g.cpu().numpy(), gr, rtol=1e-5, atol=1e-9)
