"""Ray-interval labels and the interval-guided traversal, through the C ABI.

* The label pass writes, per ray, the entry of the first and the exit of the
  last composited sample over the ray's span in the posed root; it is checked
  against the FP64 oracle's composited segments (misses: the empty interval).
* A guided render whose intervals cover every composited sample by more than a
  voxel diagonal (the exact labels with the default margin of 2 h) skips only
  empty cells, so its maps equal the plain render's bit for bit.
* The fallbacks: intervals holding no occupied voxel (F1) and intervals left
  with transmittance above the threshold (F2) both end in the full traversal,
  which again reproduces the plain maps exactly; without F2 a truncated
  interval changes the maps."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

LABEL_TOL = 1e-6


@pytest.fixture(scope="module")
def tiny2():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 2)
    K, c2w = sg.make_cameras(s, 3, 96, 112)
    rend = make_renderer(s, poses, K, c2w, 96, 112)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    return s, rend, B, K, c2w


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_labels_match_oracle(tiny2, lam):
    s, rend, B, K, c2w = tiny2
    sig, f = flut(s)
    lab = rend.proposal_labels(sig, f, lambda_th=lam).cpu().numpy()
    o, d = oracle.camera_rays(K, c2w, 96, 112)
    for p in range(B.shape[0]):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(K.shape[0]):
            log(f"labels lambda={lam} pose {p} view {v}")
            ref = oracle.render(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, ok, ol, s.sigma, s.feat, lam)
            want = oracle.interval_labels(ref["seg"])
            got = lab[p, v].reshape(-1, 2).astype(np.float64)
            # rays on the rounding guard band of the partition may differ by a sample
            band = (ref["min_gap"] < 1e-9 / (1 << s.depth)) | (ref["min_tgap"] < 1e-5)
            miss = ref["n_comp"] == 0
            assert np.array_equal(got[miss & ~band], want[miss & ~band])
            err = np.abs(got - want)[~band & ~miss]
            assert err.size == 0 or err.max() <= LABEL_TOL, err.max()
            assert np.all(got[~miss, 0] <= got[~miss, 1])


def test_guided_render_with_exact_labels_equals_plain(tiny2):
    s, rend, B, K, c2w = tiny2
    sig, f = flut(s)
    F0, A0, T0 = rend.render(sig, f, 0.01)
    lab = rend.proposal_labels(sig, f, 0.01)
    log("guided render, exact labels, margin 2h")
    F1, A1, T1 = rend.render_proposal(sig, f, lab, 0.01, margin_h=2.0)
    st = rend.stats()
    assert st["proposal_rays"] > 0
    assert st["fallbacks"] == 0
    assert np.array_equal(F0.cpu().numpy(), F1.cpu().numpy())
    assert np.array_equal(A0.cpu().numpy(), A1.cpu().numpy())
    assert np.array_equal(T0.cpu().numpy(), T1.cpu().numpy())


def test_f1_fallback_restores_plain(tiny2):
    import torch
    s, rend, B, K, c2w = tiny2
    sig, f = flut(s)
    F0, A0, _ = rend.render(sig, f, 0.01)
    # an interval at the far end of every ray, where the root holds no voxel
    iv = torch.ones((rend.P, rend.V, rend.H, rend.W, 2), dtype=torch.float32, device="cuda")
    log("guided render, intervals without voxels (F1)")
    F1, A1, _ = rend.render_proposal(sig, f, iv, 0.01, margin_h=0.5)
    st = rend.stats()
    assert st["proposal_rays"] > 0 and st["fallbacks"] == st["proposal_rays"]
    assert np.array_equal(F0.cpu().numpy(), F1.cpu().numpy())
    assert np.array_equal(A0.cpu().numpy(), A1.cpu().numpy())


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_f2_fallback_on_truncated_intervals(tiny2, lam):
    s, rend, B, K, c2w = tiny2
    sig, f = flut(s)
    F0, A0, _ = rend.render(sig, f, lam)
    lab = rend.proposal_labels(sig, f, lam)
    import torch
    trunc = lab.clone()
    hit = lab[..., 0] <= lab[..., 1]
    # rays with samples keep only the surroundings of their first sample; misses keep (1, 0)
    trunc[..., 1] = torch.where(hit, lab[..., 0], lab[..., 1])
    log(f"guided render, truncated intervals, F2 off / on, lambda={lam}")
    Fa, Aa, _ = rend.render_proposal(sig, f, trunc, lam, margin_h=0.5, f2_tau=-1.0)
    assert rend.stats()["fallbacks"] == 0
    assert not np.array_equal(F0.cpu().numpy(), Fa.cpu().numpy())
    Fb, Ab, _ = rend.render_proposal(sig, f, trunc, lam, margin_h=0.5, f2_tau=max(lam, 1e-30))
    st = rend.stats()
    assert st["fallbacks"] > 0
    assert np.array_equal(F0.cpu().numpy(), Fb.cpu().numpy())
    assert np.array_equal(A0.cpu().numpy(), Ab.cpu().numpy())


def test_predicted_empty_intervals_traverse_in_full(tiny2):
    import torch
    s, rend, B, K, c2w = tiny2
    sig, f = flut(s)
    F0, _, _ = rend.render(sig, f, 0.01)
    iv = torch.zeros((rend.P, rend.V, rend.H, rend.W, 2), dtype=torch.float32, device="cuda")
    iv[..., 0] = 1.0   # (1, 0): empty
    F1, _, _ = rend.render_proposal(sig, f, iv, 0.01)
    st = rend.stats()
    assert st["proposal_rays"] == 0 and st["fallbacks"] == 0
    assert np.array_equal(F0.cpu().numpy(), F1.cpu().numpy())


def test_proposal_argument_errors(tiny2):
    import paper_2202_05628_amd as art
    import torch
    s, rend, B, K, c2w = tiny2
    sig, f = flut(s)
    iv = torch.zeros((rend.P, rend.V, rend.H, rend.W, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(art.ArtemisError):
        rend.render_proposal(sig, f, iv, 0.01, margin_h=-1.0)
    with pytest.raises(art.ArtemisError):
        rend.render_proposal(sig, f, iv, 0.01, margin_h=float("nan"))
