"""The segmented adjoint (art_render_ckpt + art_backward_ckpt): the forward
with ray checkpoints renders the plain forward's maps bit for bit and writes
consistent records; the adjoint split into K + 1 segments per ray gives the
FP64 oracle's gradient (tiny scene, C = 8 and 16, lambda_th 0 and 0.01,
segments of 3 samples so that most rays are split several times) and, at
the differentiation workload, the unsegmented adjoint's gradient up to the
float summation order, with the same ray and sample counts."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4


@pytest.fixture(scope="module", params=[8, 16], ids=["C8", "C16"])
def tiny(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny", C=request.param)
    poses = sg.make_poses(s.J, 2)
    K, c2w = sg.make_cameras(s, 2, 96, 96)
    rend = make_renderer(s, poses, K, c2w, 96, 96)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    return s, rend, B, K, c2w


def test_checkpointed_forward_equals_forward(tiny):
    import torch
    s, rend, *_ = tiny
    sig, f = flut(s)
    F0, A0, T0 = rend.render(sig, f, 0.01)
    F, A, T, (rec, cnt, K, every) = rend.render_ckpt(sig, f, 0.01, K=6, every=3)
    assert torch.equal(F, F0) and torch.equal(A, A0) and torch.equal(T, T0)
    c = cnt.cpu().numpy()
    r = rec.cpu().numpy()
    assert c.min() >= 0 and c.max() <= K and (c > 0).sum() > 100
    # per ray: entry distances increase, T decreases, each T in (0, 1) and above the final T
    Tf = T.cpu().numpy()
    idx = np.argwhere(c >= 2)
    for p, v, y, x in idx[:: max(1, len(idx) // 400)]:
        n = c[p, v, y, x]
        t = r[p, v, y, x, :n, :2].copy().view(np.float64)[:, 0]
        Tk = r[p, v, y, x, :n, 2]
        ok_t, ok_T = np.all(np.diff(t) > 0), np.all(np.diff(Tk) < 0)
        if not (ok_t and ok_T):
            log(f"ray {(p, v, y, x)}: n {n}, t {t.tolist()}, T {Tk.tolist()}, T_final {Tf[p, v, y, x]}")
        assert ok_t and ok_T
        assert 0.0 < Tk[-1] and Tk[0] < 1.0 and Tk[-1] >= Tf[p, v, y, x]


def test_checkpoint_arguments_are_checked(tiny):
    """K outside 1..64, every outside 1..65536, a NULL or misaligned record
    buffer: ART_EINVAL before any work, and the context renders afterwards."""
    import ctypes
    import torch
    from paper_2202_05628_amd import _lib
    s, rend, *_ = tiny
    sig, f = flut(s)
    F0, A0, T0 = rend.render(sig, f, 0.01)
    F, A, T = torch.empty_like(F0), torch.empty_like(A0), torch.empty_like(T0)
    cnt = torch.zeros_like(A0, dtype=torch.int32)
    rec = torch.empty(A0.numel() * 6 * (s.C + 4) + 2, dtype=torch.float32, device="cuda")
    ds, df = torch.zeros_like(sig), torch.zeros_like(f)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    bad = [(0, 3, p(rec)), (65, 3, p(rec)), (6, 0, p(rec)), (6, 65537, p(rec)), (6, 3, None),
           (6, 3, ctypes.c_void_p(rec.data_ptr() + 4))]
    for K, every, rp in bad:
        rc = rend.lib.art_render_ckpt(rend._h, s.C, _lib.ART_F32, p(sig), p(f), 0.01, 0, p(F), p(A), p(T),
                                      K, every, rp, p(cnt))
        assert rc == _lib.ART_EINVAL, (K, every)
        rc = rend.lib.art_backward_ckpt(rend._h, s.C, _lib.ART_F32, p(sig), p(f), 0.01, 0, p(F0), p(T0), p(F0),
                                        None, p(ds), p(df), K, every, rp, p(cnt))
        assert rc == _lib.ART_EINVAL, (K, every)
    assert not ds.any() and not df.any()
    F1, A1, T1 = rend.render(sig, f, 0.01)
    assert torch.equal(F1, F0) and torch.equal(A1, A0) and torch.equal(T1, T0)


def test_checkpoints_after_tile_list_overflow(tiny, monkeypatch):
    """With tile lists too small for the call (every item renders again after
    the lists grow), the records and counts equal those of a call without
    overflow bit for bit, and the segmented adjoint from them equals the one
    from the records of the call without overflow."""
    import torch
    s, rend, B, K, c2w = tiny
    sig, f = flut(s)
    F0, A0, T0, (rec0, cnt0, _, _) = rend.render_ckpt(sig, f, 0.01, K=6, every=3)
    monkeypatch.setenv("ARTEMIS_PAIR_CAP", "64")   # every tile list overflows
    poses = sg.make_poses(s.J, 2)
    rend2 = make_renderer(s, poses, K, c2w, 96, 96)
    F, A, T, ck = rend2.render_ckpt(sig, f, 0.01, K=6, every=3)
    monkeypatch.delenv("ARTEMIS_PAIR_CAP")
    assert torch.equal(F, F0) and torch.equal(A, A0) and torch.equal(T, T0)
    c0 = cnt0.cpu().numpy()
    assert np.array_equal(ck[1].cpu().numpy(), c0)
    r0, r1 = rec0.cpu().numpy(), ck[0].cpu().numpy()
    k = np.arange(r0.shape[4])[None, None, None, None, :] < c0[..., None]   # written records
    w = s.C + 3   # t (2 words), T, P[C]; the last word is unused
    assert np.array_equal(r0[k][:, :w].view(np.uint32), r1[k][:, :w].view(np.uint32))
    rng = np.random.default_rng(9)
    dF = torch.from_numpy(rng.normal(size=tuple(F.shape)).astype(np.float32)).cuda()
    ds0, df0 = rend.backward(sig, f, F0, T0, dF, None, 0.01, ckpt=(rec0, cnt0, 6, 3))
    ds1, df1 = rend2.backward(sig, f, F, T, dF, None, 0.01, ckpt=ck, reuse_build=True)
    es = (ds1 - ds0).abs().max().item() / ds0.abs().max().item()
    ef = (df1 - df0).abs().max().item() / df0.abs().max().item()
    log(f"checkpoints after overflow: dsigma rel {es:.2e}, dfeat rel {ef:.2e}")
    assert es <= 1e-6 and ef <= 1e-6


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_segmented_adjoint_matches_oracle(tiny, lam):
    import torch
    s, rend, B, K, c2w = tiny
    rng = np.random.default_rng(5)
    target = rng.normal(size=(2, 2, s.C, 96, 96)).astype(np.float32)
    gA = rng.normal(size=(2, 2, 96, 96)).astype(np.float32)
    sig, f = flut(s)
    F, A, T, ck = rend.render_ckpt(sig, f, lam, K=6, every=3)
    dF = (F - torch.from_numpy(target).cuda()).contiguous()
    dA = torch.from_numpy(gA).cuda()
    ds, df = rend.backward(sig, f, F, T, dF, dA, lam, ckpt=ck)
    st = rend.stats()
    ds1, df1 = rend.backward(sig, f, F, T, dF, dA, lam)
    st1 = rend.stats()
    o, d = oracle.camera_rays(K, c2w, 96, 96)
    ds_ref = np.zeros(s.n)
    df_ref = np.zeros((s.n, s.C))
    for p in range(2):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(2):
            ov, dv = o[v].reshape(-1, 3), d[v].reshape(-1, 3)
            ref = oracle.render(ov, dv, s.depth, ok, ol, s.sigma, s.feat, lam)
            a, b = oracle.backward(ov, dv, s.depth, ok, ol, s.sigma, s.feat, lam,
                                   ref["F"] - target[p, v].reshape(s.C, -1).T, gA[p, v].reshape(-1))
            ds_ref += a
            df_ref += b
    ds = ds.cpu().numpy()
    df = df.cpu().numpy()
    es = np.abs(ds - ds_ref).max() / np.abs(ds_ref).max()
    ef = np.abs(df - df_ref).max() / np.abs(df_ref).max()
    e1 = np.abs(ds - ds1.cpu().numpy()).max() / np.abs(ds_ref).max()
    log(f"segmented adjoint C = {s.C}, lambda {lam}: dsigma rel_max {es:.2e}, dfeat rel_max {ef:.2e}, "
        f"vs unsegmented {e1:.2e}; rounds {st['rounds']} (unsegmented {st1['rounds']})")
    assert es <= TOL_GRAD and ef <= TOL_GRAD
    assert np.all(ds[ds_ref == 0] == 0)
    for k in ("rays", "samples", "hit_rays", "tile_rays"):
        assert st[k] == st1[k], k


def test_segmented_adjoint_full_scale(monkeypatch):
    """The differentiation workload (full scene, 1 pose x 4 cameras at 512^2,
    C = 16): segments of 32 samples, K = 8."""
    import torch
    cfg = sg.CONFIGS["grad"]
    s = sg.make_scene(cfg)
    poses = sg.make_poses(s.J, cfg.n_poses, cfg.pose_seed0)
    K, c2w = sg.make_cameras(s, cfg.n_views, cfg.height, cfg.width)
    rend = make_renderer(s, poses, K, c2w, cfg.height, cfg.width)
    sig, f = flut(s)
    F, A, T, ck = rend.render_ckpt(sig, f, 0.01, K=8, every=32)
    tgt = torch.from_numpy(sg.make_targets(1, cfg.n_views, s.C, cfg.height, cfg.width, cfg.target_seed)).cuda()
    dF = (F - tgt).contiguous()
    out = {}
    for mode in ("segmented", "whole"):
        for merge in ("0", "1"):
            monkeypatch.setenv("ARTEMIS_ADJ_MERGE", merge)
            ds, df = rend.backward(sig, f, F, T, dF, None, 0.01, ckpt=ck if mode == "segmented" else None,
                                   reuse_build=True)
            out[(mode, merge)] = (ds.cpu().numpy().astype(np.float64), df.cpu().numpy().astype(np.float64),
                                  rend.stats())
    ref_s, ref_f, st0 = out[("whole", "0")]
    for key, (ds, df, st) in out.items():
        es = np.abs(ds - ref_s).max() / np.abs(ref_s).max()
        ef = np.abs(df - ref_f).max() / np.abs(ref_f).max()
        log(f"full scale {key}: dsigma rel {es:.2e}, dfeat rel {ef:.2e}, rounds {st['rounds']}, "
            f"samples {st['samples']}")
        assert es <= 1e-5 and ef <= 1e-5
        assert st["samples"] == st0["samples"] and st["rays"] == st0["rays"]
        assert np.array_equal(ds != 0, ref_s != 0)
