"""View-dependent features (Eq. 2 inside Eq. 5) through the C ABI, against the
FP64 oracle's render_sh on the same seeded inputs.

The FLUT holds H real-SH coefficient blocks of C channels per leaf; a sample
contributes w sum_h k_h Y_h(R^T d) with R the rotation of the leaf's dominant
bone.  The GPU evaluates d^c and Y in FP32 from the FP32 bone transforms, so
the maps are compared at the FP32 bar (1e-5 of the map's largest value);
opacity and transmittance do not depend on the features and equal the plain
render's bit for bit.  Rays on the rounding guard band are excluded as in the
other parity tests."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import log, make_renderer

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def tiny2():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 2)
    H, W = 60, 52
    K, c2w = sg.make_cameras(s, 2, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    return s, rend, B, K, c2w, H, W


def _sh_feat(s, nsh, C, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(s.n, nsh, C)).astype(np.float32)


# C = 16 is the channel count of the full workload (its kernels are their own
# template instances)
@pytest.mark.parametrize("nsh,storage,C", [(1, "f32", 8), (4, "f32", 8), (9, "f32", 8), (9, "bf16", 8),
                                           (9, "f32", 16), (9, "bf16", 16)])
def test_sh_render_matches_oracle(tiny2, nsh, storage, C):
    import torch
    s, rend, B, K, c2w, H, W = tiny2
    k = _sh_feat(s, nsh, C, 30 + nsh + C)
    sig = torch.from_numpy(s.sigma).cuda()
    f = torch.from_numpy(k).cuda()
    if storage == "bf16":
        sig, f = sig.to(torch.bfloat16), f.to(torch.bfloat16)
    sig_np = sig.float().cpu().numpy().astype(np.float64)
    k_np = f.float().cpu().numpy().astype(np.float64)
    F, A, T = rend.render_sh(sig.contiguous(), f.contiguous(), 0.01)
    _, A0, T0 = rend.render(sig.contiguous(), f[:, 0, :].contiguous(), 0.01)
    assert np.array_equal(A.cpu().numpy(), A0.cpu().numpy())
    assert np.array_equal(T.cpu().numpy(), T0.cpu().numpy())
    dom = oracle.dominant_bone(s.bone, s.weight)
    o, d = oracle.camera_rays(K, c2w, H, W)
    Fn = F.cpu().numpy()
    worst = 0.0
    for p in range(B.shape[0]):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(K.shape[0]):
            ref = oracle.render_sh(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, ok, ol, sig_np, k_np, nsh,
                                   dom, B[p], 0.01)
            band = (ref["min_gap"] < 1e-9 / (1 << s.depth)) | (ref["min_tgap"] < 1e-5)
            got = Fn[p, v].reshape(Fn.shape[2], -1).T
            err = np.abs(got - ref["F"])[~band].max() / np.abs(ref["F"]).max()
            worst = max(worst, err)
    log(f"SH H={nsh} C={C} {storage}: rel_max {worst:.2e}")
    assert worst <= TOL


def test_sh_degree0_is_the_plain_render_scaled(tiny2):
    import torch
    s, rend, B, K, c2w, H, W = tiny2
    sig = torch.from_numpy(s.sigma).cuda()
    f = torch.from_numpy(s.feat).cuda()
    F1, _, _ = rend.render_sh(sig, f[:, None, :].contiguous(), 0.01)
    F0, _, _ = rend.render(sig, f, 0.01)
    y0 = 0.5 / math.sqrt(math.pi)
    err = float((F1 - y0 * F0).abs().max() / (y0 * F0).abs().max())
    assert err <= 1e-6


def test_sh_argument_errors(tiny2):
    import paper_2202_05628_amd as art
    import torch
    s, rend, B, K, c2w, H, W = tiny2
    sig = torch.from_numpy(s.sigma).cuda()
    f = torch.zeros((s.n, 2, s.feat.shape[1]), dtype=torch.float32, device="cuda")
    with pytest.raises(art.ArtemisError):
        rend.render_sh(sig, f, 0.01)
