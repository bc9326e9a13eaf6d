"""GPU adjoint (the hand-written backward compositing kernel behind the
autograd Function) against the FP64 oracle's gradient and central finite
differences of the FP64 oracle."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4


# C = 16 and 32 map 4 and 2 samples onto one atomic instruction of the
# adjoint's row-wise gradient scatter, C = 8 eight: each is its own code path
@pytest.fixture(scope="module", params=[8, 16, 32], ids=["C8", "C16", "C32"])
def tiny(request):
    s = sg.make_scene("tiny", C=request.param)
    poses = sg.make_poses(s.J, 2)
    K, c2w = sg.make_cameras(s, 2, 96, 96)
    rend = make_renderer(s, poses, K, c2w, 96, 96)
    B = oracle.fk(s.parent, s.rest_joint, *poses)
    return s, rend, B, K, c2w


def _oracle_grad(s, B, K, c2w, H, W, lam, target, gA):
    o, d = oracle.camera_rays(K, c2w, H, W)
    ds = np.zeros(s.n)
    df = np.zeros((s.n, s.C))
    F_all = []
    for p in range(B.shape[0]):
        ok, ol, _, _, _ = oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])
        for v in range(K.shape[0]):
            ov, dv = o[v].reshape(-1, 3), d[v].reshape(-1, 3)
            ref = oracle.render(ov, dv, s.depth, ok, ol, s.sigma, s.feat, lam)
            g = ref["F"] - target[p, v].reshape(s.C, -1).T
            a, b = oracle.backward(ov, dv, s.depth, ok, ol, s.sigma, s.feat, lam, g,
                                   gA[p, v].reshape(-1))
            ds += a
            df += b
            F_all.append(ref)
    return ds, df, F_all


@pytest.mark.parametrize("merge", ["default", "merged"])
@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_adjoint_matches_oracle(tiny, lam, merge, monkeypatch):
    """merge: the records of one leaf summed before the atomics (forced; by
    default a launch this small adds them in buffer order)."""
    import torch
    import paper_2202_05628_amd as art

    if merge == "merged":
        monkeypatch.setenv("ARTEMIS_ADJ_MERGE", "1")
    s, rend, B, K, c2w = tiny
    rng = np.random.default_rng(3)
    target = rng.normal(size=(2, 2, s.C, 96, 96)).astype(np.float32)
    gA = rng.normal(size=(2, 2, 96, 96)).astype(np.float32)
    sig, f = flut(s)
    sig.requires_grad_(True)
    f.requires_grad_(True)
    log(f"adjoint: tiny, C = {s.C}, 2 poses x 2 views, lambda {lam}")
    F, A = art.render(rend, sig, f, lambda_th=lam)
    tgt = torch.from_numpy(target).cuda()
    loss = 0.5 * ((F - tgt) ** 2).sum() + (A * torch.from_numpy(gA).cuda()).sum()
    loss.backward()
    ds_ref, df_ref, _ = _oracle_grad(s, B, K, c2w, 96, 96, lam, target, gA)
    ds = sig.grad.cpu().numpy()
    df = f.grad.cpu().numpy()
    es = np.abs(ds - ds_ref).max() / np.abs(ds_ref).max()
    ef = np.abs(df - df_ref).max() / np.abs(df_ref).max()
    st = rend.stats()
    log(f"  {merge}: dsigma rel_max {es:.2e}, dfeat rel_max {ef:.2e}; "
        f"{st['grad_adds']} gradient additions for {st['samples']} samples")
    assert es <= TOL_GRAD and ef <= TOL_GRAD
    # hidden leaves and collision losers get exactly zero
    assert np.all(ds[ds_ref == 0] == 0)
    if merge == "default":
        assert st["grad_adds"] == st["samples"]
    else:
        assert st["grad_adds"] < st["samples"]


def test_adjoint_against_finite_differences(tiny):
    """GPU gradient vs central differences (h = 1e-3) of the FP64 oracle on 64
    random visible leaves (lambda_th = 0: no stop sample moves)."""
    import torch

    s, rend, B, K, c2w = tiny
    rng = np.random.default_rng(9)
    target = rng.normal(size=(2, 2, s.C, 96, 96)).astype(np.float32)
    sig, f = flut(s)
    F, A, T = rend.render(sig, f, lambda_th=0.0)
    dF = F - torch.from_numpy(target).cuda()
    ds, df = rend.backward(sig, f, F, T, dF, None, lambda_th=0.0)
    ds = ds.cpu().numpy()
    df = df.cpu().numpy()
    o, d = oracle.camera_rays(K, c2w, 96, 96)
    occ = [oracle.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B[p])[:2] for p in range(2)]
    # the oracle's own hit lists tell which rays each leaf touches; the loss
    # changes only through those rays
    hits = {}
    for p in range(2):
        for v in range(2):
            r = oracle.render(o[v].reshape(-1, 3), d[v].reshape(-1, 3), s.depth, occ[p][0], occ[p][1],
                              s.sigma, s.feat, 0.0, max_hits=256)
            assert r["n_comp"].max() <= 256
            hits[(p, v)] = r["hit_leaf"]

    def loss(sigma, feat, leaf):
        L = 0.0
        for (p, v), hl in hits.items():
            rays = np.flatnonzero((hl == leaf).any(axis=1))
            if len(rays) == 0:
                continue
            r = oracle.render(o[v].reshape(-1, 3)[rays], d[v].reshape(-1, 3)[rays], s.depth, occ[p][0],
                              occ[p][1], sigma, feat, 0.0)
            L += 0.5 * np.sum((r["F"] - target[p, v].reshape(s.C, -1).T[rays]) ** 2)
        return L

    vis = np.flatnonzero(ds != 0)
    pick = rng.choice(vis, 64, replace=False)
    sigma = s.sigma.astype(np.float64)
    feat = s.feat.astype(np.float64)
    eps = 1e-3
    scale_s = np.abs(ds).max()
    scale_f = np.abs(df).max()
    for leaf in pick:
        sp = sigma.copy(); sp[leaf] += eps
        sm = sigma.copy(); sm[leaf] -= eps
        fd = (loss(sp, feat, leaf) - loss(sm, feat, leaf)) / (2 * eps)
        assert abs(fd - ds[leaf]) <= TOL_GRAD * scale_s, (leaf, fd, ds[leaf])
        c = int(rng.integers(0, s.C))
        fp = feat.copy(); fp[leaf, c] += eps
        fm = feat.copy(); fm[leaf, c] -= eps
        fd = (loss(sigma, fp, leaf) - loss(sigma, fm, leaf)) / (2 * eps)
        assert abs(fd - df[leaf, c]) <= TOL_GRAD * scale_f, (leaf, c, fd, df[leaf, c])
