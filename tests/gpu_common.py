"""Shared helpers of the GPU parity tests: build a renderer for a scene and
compute the oracle's reference for the same seeded inputs."""
import math
import sys

import numpy as np

import oracle
import scenegen as sg


def log(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)


def make_renderer(scene, poses, K, c2w, H, W):
    import paper_2202_05628_amd as art
    r = art.Renderer(0)
    r.set_scene(scene)
    r.set_poses(*poses)
    r.set_cameras(K, c2w, H, W)
    return r


def flut(scene, dtype="f32"):
    import torch
    sig = torch.from_numpy(scene.sigma).cuda()
    f = torch.from_numpy(scene.feat).cuda()
    if dtype == "bf16":
        return sig.to(torch.bfloat16), f.to(torch.bfloat16)
    return sig.contiguous(), f.contiguous()


def guard_leaves(pt, depth, eps=1e-9):
    """Leaves whose posed centre lies within eps*h of a lattice plane."""
    u = (pt + 1.0) * (1 << depth)
    frac = np.abs(u - np.round(u))
    return np.any(frac < eps, axis=1)


def oracle_pose(scene, B_pose):
    return oracle.pose_occupancy(scene.ijk, scene.depth, scene.bone, scene.weight, B_pose)


def oracle_maps(scene, B, K, c2w, H, W, lam, sigma=None, feat=None, pixels=None, max_hits=0):
    """Oracle F [P][V][C][H*W or k], A, T, flags for all poses/views (or a pixel subset)."""
    sigma = scene.sigma if sigma is None else sigma
    feat = scene.feat if feat is None else feat
    o, d = oracle.camera_rays(K, c2w, H, W)
    V = K.shape[0]
    out = []
    for p in range(B.shape[0]):
        ok, ol, _, _, _ = oracle_pose(scene, B[p])
        per_view = []
        for v in range(V):
            ov = o[v].reshape(-1, 3)
            dv = d[v].reshape(-1, 3)
            if pixels is not None:
                ov, dv = ov[pixels], dv[pixels]
            per_view.append(oracle.render(ov, dv, scene.depth, ok, ol, sigma, feat, lam, max_hits=max_hits))
        out.append(per_view)
    return out


def map_error(F_gpu, F_ref, mask=None):
    """rel_max / rel_mean of one map (optionally restricted to a pixel mask)."""
    if mask is not None:
        F_gpu = F_gpu[..., mask]
        F_ref = F_ref[..., mask]
    return oracle.map_rel_error(F_gpu, F_ref)
