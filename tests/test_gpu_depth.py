"""The depth buffer of hybrid rendering (Section 3.1, paragraph "Hybrid
Rendering") through the C ABI.

Per pixel: the distance along the ray to the entry of the first occupied voxel
whose density is above a threshold, searched along the whole ray whether or not
the compositing stopped early (+inf if none), against the FP64 oracle on the
same seeded scene.  The threshold decision is taken on the
stored density on both sides (FP32 or BF16 values, a threshold representable
in FP32), so the set of counted samples is exact; the distance is compared to
FP32 rounding.  The maps written beside the depth equal art_render's bit for
bit.  Rays on the rounding guard band of the partition (a lattice crossing
within 1e-9 h of another) or of the early stop (transmittance within 1e-5 of
the threshold) may differ by a sample and are excluded, as in the other
parity tests."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

DEPTH_TOL = 1e-6   # relative, FP32 rounding of an FP64 distance


@pytest.fixture(scope="module", params=[(96, 112), (90, 102)], ids=["96x112", "90x102"])
def tiny2(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    H, W = request.param
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 2)
    K, c2w = sg.make_cameras(s, 3, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    return s, rend, B, K, c2w, H, W


def _check(s, B, K, c2w, H, W, lam, sig_np, feat_np, th, D):
    o, d = oracle.camera_rays(K, c2w, H, W)
    n_fin = 0
    for p in range(B.shape[0]):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(K.shape[0]):
            ref = oracle.render(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, ok, ol, sig_np, feat_np, lam,
                                depth_sigma=th)
            want = ref["dist"]
            got = D[p, v].reshape(-1).astype(np.float64)
            band = (ref["min_gap"] < 1e-9 / (1 << s.depth)) | (ref["min_tgap"] < 1e-5)
            inf_w = np.isinf(want)
            assert np.array_equal(np.isinf(got)[~band], inf_w[~band]), (p, v)
            fin = ~band & ~inf_w
            if fin.any():
                err = np.abs(got[fin] - want[fin]) / np.abs(want[fin])
                assert err.max() <= DEPTH_TOL, (p, v, err.max())
            n_fin += int(fin.sum())
    return n_fin


@pytest.mark.parametrize("lam", [0.0, 0.01])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_depth_matches_oracle(tiny2, lam, storage):
    import torch
    s, rend, B, K, c2w, H, W = tiny2
    sig, f = flut(s, storage)
    sig_np = sig.float().cpu().numpy().astype(np.float64)
    feat_np = f.float().cpu().numpy().astype(np.float64)
    th = float(np.float32(np.median(sig_np)))
    log(f"depth {H}x{W} {storage} lambda={lam} threshold={th:.4f}")
    F0, A0, T0 = rend.render(sig, f, lam)
    F1, A1, T1, D = rend.render_depth(sig, f, th, lam)
    assert np.array_equal(F0.cpu().numpy(), F1.cpu().numpy())
    assert np.array_equal(A0.cpu().numpy(), A1.cpu().numpy())
    assert np.array_equal(T0.cpu().numpy(), T1.cpu().numpy())
    n_fin = _check(s, B, K, c2w, H, W, lam, sig_np, feat_np, th, D.cpu().numpy())
    log(f"  {n_fin} finite depths checked")
    assert n_fin > 100


def test_depth_threshold_extremes(tiny2):
    """A threshold below every density gives the entry of the first composited
    sample (the label pass's u_near mapped back to a distance); one above every
    density gives +inf everywhere."""
    import torch
    s, rend, B, K, c2w, H, W = tiny2
    sig, f = flut(s)
    _, A, _, D = rend.render_depth(sig, f, -1.0, 0.01)
    hit = (A > 0).cpu().numpy()
    Dn = D.cpu().numpy()
    assert np.all(np.isfinite(Dn[hit])) and np.all(Dn[hit] > 0)
    assert np.all(np.isinf(Dn[~hit]))
    _, _, _, D2 = rend.render_depth(sig, f, 3.0e38, 0.01)
    assert torch.isinf(D2).all()


def test_depth_argument_errors(tiny2):
    import paper_2202_05628_amd as art
    s, rend, B, K, c2w, H, W = tiny2
    sig, f = flut(s)
    with pytest.raises(art.ArtemisError):
        rend.render_depth(sig, f, float("nan"), 0.01)


@pytest.mark.parametrize("C", [8, 16])
def test_depth_past_the_early_stop(C):
    """A threshold above most densities: many rays turn opaque (T < 0.01)
    before they reach a voxel above it, and their depth lies beyond the last
    composited sample; the kernel's depth-only scan past the stop must find it."""
    import torch
    s = sg.make_scene("tiny", C=C)
    poses = sg.make_poses(s.J, 2)
    H, W = 90, 102
    K, c2w = sg.make_cameras(s, 2, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    sig, f = flut(s)
    sig_np = sig.cpu().numpy().astype(np.float64)
    th = float(np.float32(np.quantile(sig_np, 0.97)))
    log(f"depth past the stop: C = {C}, threshold {th:.3f}")
    F0, A0, T0 = rend.render(sig, f, 0.01)
    F1, A1, T1, D = rend.render_depth(sig, f, th, 0.01)
    assert np.array_equal(F0.cpu().numpy(), F1.cpu().numpy())
    assert np.array_equal(A0.cpu().numpy(), A1.cpu().numpy())
    assert np.array_equal(T0.cpu().numpy(), T1.cpu().numpy())
    n_fin = _check(s, B, K, c2w, H, W, 0.01, sig_np, s.feat.astype(np.float64), th, D.cpu().numpy())
    o, d = oracle.camera_rays(K, c2w, H, W)
    late = 0
    for p in range(2):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(2):
            ref = oracle.render(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, ok, ol, sig_np,
                                s.feat.astype(np.float64), 0.01, depth_sigma=th)
            late += int((np.isfinite(ref["dist"]) & (ref["dist"] >= ref["seg"][:, 3])).sum())
    log(f"  {n_fin} finite depths checked, {late} of them beyond the early stop")
    assert late > 100
