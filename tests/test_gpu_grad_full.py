"""The adjoint at the differentiation workload: the full scene (1.5M leaves,
40 bones, C = 16), one pose (seed 1000), 4 cameras at 512x512, lambda_th =
0.01, in the launch configuration the benchmark's adjoint leg times.

The loss is L = 1/2 sum (F - F*)^2 over a seeded subset of 20,000 rays (the
map gradient dL/dF = F - F* on those rays, 0 elsewhere), F* ~ N(0, 1), so the
FP64 oracle's gradient needs only those rays.  Checked:

* the GPU's dL/dsigma and dL/df over every leaf against the oracle's
  gradient (rel_max over the whole gradient vectors, 1e-4);
* central finite differences (h = 1e-3) of the FP64 oracle's loss at 64
  random leaves with a non-zero gradient, against the oracle's own gradient
  (1e-6 of the largest entry: a pin of the oracle) and the GPU's (1e-4).

The subset holds rays away from the rounding guard bands (no lattice crossing
within 1e-9 h of another, transmittance at every step farther than 1e-5
relative from lambda_th), where the two sides may composite a different
sample list.  A finite difference whose perturbation changes the composited
sample count of a ray (a stop sample that moves) is not used."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4
TOL_FD_ORACLE = 1e-6
LAM = 0.01
N_RAYS = 20_000


@pytest.fixture(scope="module")
def grad_full():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("grad")
    cfg = sg.CONFIGS["grad"]
    poses = sg.make_poses(s.J, cfg.n_poses, cfg.pose_seed0)
    H, W, V = cfg.height, cfg.width, cfg.n_views
    K, c2w = sg.make_cameras(s, V, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[0])
    o, d = oracle.camera_rays(K, c2w, H, W)
    o = o.reshape(-1, 3)
    d = d.reshape(-1, 3)
    target = sg.make_targets(1, V, s.C, H, W, seed=cfg.target_seed)[0]   # [V][C][H][W]
    tgt_rays = np.moveaxis(target.reshape(V, s.C, H * W), 1, 2).reshape(-1, s.C)   # [V*H*W][C]
    # the subset: seeded candidates, half from rays the oracle sees hit something
    rng = np.random.default_rng(1000)
    cand = rng.choice(V * H * W, 6 * N_RAYS, replace=False)
    ref = oracle.render(o[cand], d[cand], s.depth, ok, ol, s.sigma, s.feat, LAM)
    h = 1.0 / (1 << s.depth)
    good = (ref["min_gap"] >= 1e-9 * h) & (ref["min_tgap"] >= 1e-5)
    hit = good & (ref["n_comp"] > 0)
    miss = good & (ref["n_comp"] == 0)
    sub = np.sort(np.concatenate([cand[hit][: N_RAYS // 2], cand[miss][: N_RAYS - min(hit.sum(), N_RAYS // 2)]]))
    assert len(sub) == N_RAYS
    log(f"grad-full: {len(sub)} rays in the loss ({int(hit.sum())} good hit candidates)")
    return s, rend, ok, ol, o, d, tgt_rays, sub


def _gpu_grad(s, rend, tgt_rays, sub, H, W, V):
    import torch
    sig, f = flut(s)
    F, A, T = rend.render(sig, f, lambda_th=LAM)
    Fr = F[0].permute(0, 2, 3, 1).reshape(-1, s.C)   # [V*H*W][C]
    g = torch.zeros_like(Fr)
    idx = torch.from_numpy(sub).cuda()
    g[idx] = Fr[idx] - torch.from_numpy(tgt_rays[sub]).cuda()
    dF = g.reshape(1, V, H, W, s.C).permute(0, 1, 4, 2, 3).contiguous()
    ds, df = rend.backward(sig, f, F, T, dF, None, lambda_th=LAM, reuse_build=True)
    return ds.cpu().numpy().astype(np.float64), df.cpu().numpy().astype(np.float64)


def test_adjoint_full_matches_oracle(grad_full, monkeypatch):
    """Both ways the adjoint adds its gradients: records in buffer order (the
    default at this workload, which has fewer tiles than workgroups) and the
    records of one leaf merged first (forced)."""
    s, rend, ok, ol, o, d, tgt_rays, sub = grad_full
    cfg = sg.CONFIGS["grad"]
    ref = oracle.render(o[sub], d[sub], s.depth, ok, ol, s.sigma, s.feat, LAM)
    ds_ref, df_ref = oracle.backward(o[sub], d[sub], s.depth, ok, ol, s.sigma, s.feat, LAM,
                                     ref["F"] - tgt_rays[sub])
    touched = int((ds_ref != 0).sum())
    assert touched > 10_000
    for mode in ("default", "merged"):
        if mode == "merged":
            monkeypatch.setenv("ARTEMIS_ADJ_MERGE", "1")
        ds, df = _gpu_grad(s, rend, tgt_rays, sub, cfg.height, cfg.width, cfg.n_views)
        st = rend.stats()
        es = np.abs(ds - ds_ref).max() / np.abs(ds_ref).max()
        ef = np.abs(df - df_ref).max() / np.abs(df_ref).max()
        log(f"  {mode}: {touched} leaves with a gradient; dsigma rel_max {es:.2e}, dfeat rel_max {ef:.2e}; "
            f"{st['grad_adds']} gradient additions for {st['samples']} samples")
        assert es <= TOL_GRAD and ef <= TOL_GRAD
        # leaves no ray of the subset composites get exactly zero
        assert np.all(ds[ds_ref == 0] == 0) and np.all(df[df_ref == 0] == 0)
        if mode == "default":
            assert st["grad_adds"] == st["samples"]
        else:
            assert st["grad_adds"] < 0.9 * st["samples"]


def test_adjoint_full_finite_differences(grad_full):
    s, rend, ok, ol, o, d, tgt_rays, sub = grad_full
    cfg = sg.CONFIGS["grad"]
    ds, df = _gpu_grad(s, rend, tgt_rays, sub, cfg.height, cfg.width, cfg.n_views)
    sigma = s.sigma.astype(np.float64)
    feat = s.feat.astype(np.float64)
    ref = oracle.render(o[sub], d[sub], s.depth, ok, ol, sigma, feat, LAM, max_hits=2048)
    assert ref["n_comp"].max() <= 2048
    ds_ref, df_ref = oracle.backward(o[sub], d[sub], s.depth, ok, ol, sigma, feat, LAM, ref["F"] - tgt_rays[sub])
    hl = ref["hit_leaf"]
    rng = np.random.default_rng(64)
    pick = rng.choice(np.flatnonzero(ds_ref != 0), 64, replace=False)
    eps = 1e-3
    sc_s, sc_f = np.abs(ds_ref).max(), np.abs(df_ref).max()

    def loss(sg_, ft_, rays):
        r = oracle.render(o[sub][rays], d[sub][rays], s.depth, ok, ol, sg_, ft_, LAM)
        return 0.5 * np.sum((r["F"] - tgt_rays[sub][rays]) ** 2), r["n_comp"]

    used = 0
    for leaf in pick:
        rays = np.flatnonzero((hl == leaf).any(axis=1))
        assert len(rays) > 0
        n0 = ref["n_comp"][rays]
        sp = sigma.copy(); sp[leaf] += eps
        sm = sigma.copy(); sm[leaf] -= eps
        lp, np_ = loss(sp, feat, rays)
        lm, nm = loss(sm, feat, rays)
        if np.array_equal(np_, n0) and np.array_equal(nm, n0):   # no stop sample moved
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - ds_ref[leaf]) <= TOL_FD_ORACLE * sc_s, (leaf, fd, ds_ref[leaf])
            assert abs(fd - ds[leaf]) <= TOL_GRAD * sc_s, (leaf, fd, ds[leaf])
            used += 1
        c = int(rng.integers(0, s.C))
        fp = feat.copy(); fp[leaf, c] += eps
        fm = feat.copy(); fm[leaf, c] -= eps
        fd = (loss(sigma, fp, rays)[0] - loss(sigma, fm, rays)[0]) / (2 * eps)
        assert abs(fd - df_ref[leaf, c]) <= TOL_FD_ORACLE * sc_f, (leaf, c, fd, df_ref[leaf, c])
        assert abs(fd - df[leaf, c]) <= TOL_GRAD * sc_f, (leaf, c, fd, df[leaf, c])
    log(f"  density differences used at {used} of 64 leaves")
    assert used >= 48
