"""MI355X animated-octree feature renderer (ARTEMIS, Luo et al. 2022, Section 3.1).

Python front end of libartemis.so: marshals numpy arrays and torch tensors
into the C ABI (include/artemis.h).  The skinning, octree rebuild, ray
indexing, compositing and adjoint all run in the library's HIP kernels;
PyTorch only supplies device memory and the stream.

    r = Renderer()
    r.load_octree(depth, ijk); r.set_skin(bone, weight)
    r.set_skeleton(parent, rest_joint); r.set_poses(rot, R, T)
    r.set_cameras(K, c2w, H, W)
    feat_map, alpha, t_final = r.render(sigma, feat)          # sigma [n], feat [n][C] on cuda
    feat_map, alpha = render(r, sigma, feat)                  # differentiable (autograd)
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

from . import _lib
from ._lib import ART_BF16, ART_F32, ART_GEOM_FP32, ART_PROPOSAL_MARGIN_H, ART_TIMING, ArtemisError

__all__ = ["Renderer", "render", "RenderFn", "ArtemisError", "ART_GEOM_FP32", "ART_TIMING",
           "LAMBDA_TH"]

# early-stop threshold of the paper (Section 3.1): stop once alpha > 1 - 0.01
LAMBDA_TH = 0.01


def _np(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Renderer:
    """One library context bound to a CUDA (HIP) device and the torch stream
    current at construction."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self._torch = torch
        self.lib = _lib.load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.art_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise ArtemisError(rc, f"art_create(device={device}) failed")
        self._h = h
        self.n = 0
        self.depth = 0
        self.J = 0
        self.P = 0
        self.V = self.H = self.W = 0

    # ---- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.art_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state_version(self) -> int:
        """Counter of the octree / skin / skeleton / poses / cameras setters."""
        return int(self.lib.art_state_version(self._h))

    def set_memory_limit(self, nbytes: int) -> None:
        """Bound the library's working device memory (0: no bound)."""
        self._check(self.lib.art_set_memory_limit(self._h, int(nbytes)), "art_set_memory_limit")

    def memory(self) -> dict:
        held = ctypes.c_int64(0)
        lim = ctypes.c_int64(0)
        self._check(self.lib.art_get_memory(self._h, ctypes.byref(held), ctypes.byref(lim)), "art_get_memory")
        return {"working_bytes": int(held.value), "limit": int(lim.value)}

    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = self.lib.art_last_error(self._h)
            raise ArtemisError(rc, f"{what}: {msg.decode() if msg else ''}")

    # ---- inputs -----------------------------------------------------------------
    def load_octree(self, depth: int, ijk) -> None:
        ijk = _np(ijk, np.uint16)
        self._check(self.lib.art_load_octree(self._h, int(depth), int(ijk.shape[1]), _ptr(ijk)),
                    "art_load_octree")
        self.n, self.depth = int(ijk.shape[1]), int(depth)

    def set_skin(self, bone, weight) -> None:
        b = _np(bone, np.uint8)
        w = _np(weight, np.float32)
        self._check(self.lib.art_set_skin(self._h, _ptr(b), _ptr(w)), "art_set_skin")

    def set_skeleton(self, parent, rest_joint) -> None:
        p = _np(parent, np.int32)
        r = _np(rest_joint, np.float64)
        self._check(self.lib.art_set_skeleton(self._h, int(p.shape[0]), _ptr(p), _ptr(r)),
                    "art_set_skeleton")
        self.J = int(p.shape[0])

    def set_poses(self, r, R, T) -> None:
        r = _np(r, np.float64)
        P = int(r.shape[0])
        R = _np(R, np.float64).reshape(P, 3)
        T = _np(T, np.float64).reshape(P, 3)
        self._check(self.lib.art_set_poses(self._h, P, _ptr(r), _ptr(R), _ptr(T)), "art_set_poses")
        self.P = P

    def set_cameras(self, K, c2w, H: int, W: int) -> None:
        K = _np(K, np.float64)
        c = _np(c2w, np.float64)
        V = int(K.shape[0])
        self._check(self.lib.art_set_cameras(self._h, V, int(H), int(W), _ptr(K), _ptr(c)),
                    "art_set_cameras")
        self.V, self.H, self.W = V, int(H), int(W)

    def set_scene(self, scene) -> None:
        """Load a scenegen.Scene (octree, skin, skeleton)."""
        self.load_octree(scene.depth, scene.ijk)
        self.set_skin(scene.bone, scene.weight)
        self.set_skeleton(scene.parent, scene.rest_joint)

    # ---- helpers ----------------------------------------------------------------
    def _flut(self, sigma, feat):
        torch = self._torch
        if sigma.dtype != feat.dtype or sigma.dtype not in (torch.float32, torch.bfloat16):
            raise TypeError("sigma and feat must both be float32 or both bfloat16")
        if not (sigma.is_cuda and feat.is_cuda):
            raise TypeError("sigma and feat must be device tensors")
        if sigma.shape != (self.n,) or feat.dim() != 2 or feat.shape[0] != self.n:
            raise ValueError(f"expected sigma [{self.n}] and feat [{self.n}, C]")
        if not (sigma.is_contiguous() and feat.is_contiguous()):
            raise ValueError("sigma and feat must be contiguous")
        dtype = ART_BF16 if sigma.dtype == torch.bfloat16 else ART_F32
        return int(feat.shape[1]), dtype

    def _flags(self, fp32_geom: bool, timing: bool, sync: bool = True) -> int:
        return (ART_GEOM_FP32 if fp32_geom else 0) | (ART_TIMING if timing else 0) | (0 if sync else _lib.ART_ASYNC)

    # ---- rendering ------------------------------------------------------------------
    def render(self, sigma, feat, lambda_th: float = LAMBDA_TH, fp32_geom: bool = False,
               timing: bool = False, out=None, want_tfinal: bool = True, sync: bool = True):
        """Feature maps [P][V][C][H][W], opacity [P][V][H][W], final transmittance
        [P][V][H][W] (or None) for every pose and camera.  sync=False: the call
        only enqueues the work (ART_ASYNC); render_status() reports overflows
        and invalid densities afterwards."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        dev = sigma.device
        if out is None:
            F = torch.empty((self.P, self.V, C, self.H, self.W), dtype=torch.float32, device=dev)
            A = torch.empty((self.P, self.V, self.H, self.W), dtype=torch.float32, device=dev)
            T = torch.empty_like(A) if want_tfinal else None
        else:
            F, A, T = out
        self._check(self.lib.art_render(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                        self._flags(fp32_geom, timing, sync), _tptr(F), _tptr(A), _tptr(T)),
                    "art_render")
        return F, A, T

    def render_ckpt(self, sigma, feat, lambda_th: float = LAMBDA_TH, K: int = 8, every: int = 32,
                    fp32_geom: bool = False, timing: bool = False, sync: bool = True):
        """render() that also records ray checkpoints for backward(ckpt=...)
        (art_render_ckpt): returns (F, A, T, ckpt) with ckpt = (records
        [P][V][H][W][K][C + 4] float32, counts [P][V][H][W] int32, K, every).
        sync=False: as render(sync=False)."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        dev = sigma.device
        F = torch.empty((self.P, self.V, C, self.H, self.W), dtype=torch.float32, device=dev)
        A = torch.empty((self.P, self.V, self.H, self.W), dtype=torch.float32, device=dev)
        T = torch.empty_like(A)
        rec = torch.empty((self.P, self.V, self.H, self.W, K, C + 4), dtype=torch.float32, device=dev)
        cnt = torch.zeros((self.P, self.V, self.H, self.W), dtype=torch.int32, device=dev)
        self._check(self.lib.art_render_ckpt(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                             self._flags(fp32_geom, timing, sync), _tptr(F), _tptr(A), _tptr(T),
                                             int(K), int(every), _tptr(rec), _tptr(cnt)), "art_render_ckpt")
        return F, A, T, (rec, cnt, int(K), int(every))

    def render_status(self) -> dict:
        """Outcome of the last call made with sync=False (art_render_status):
        overflowed (pose, view group) items and invalid densities."""
        ov = ctypes.c_int64(0)
        bad = ctypes.c_int64(0)
        self._check(self.lib.art_render_status(self._h, ctypes.byref(ov), ctypes.byref(bad)), "art_render_status")
        return {"overflowed_items": int(ov.value), "bad_densities": int(bad.value)}

    def render_depth(self, sigma, feat, depth_sigma: float, lambda_th: float = LAMBDA_TH, fp32_geom: bool = False,
                     timing: bool = False, out=None, want_tfinal: bool = True):
        """render() plus the depth buffer [P][V][H][W]: distance along the ray to
        the entry of the first composited sample with density > depth_sigma
        (+inf if none)."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        dev = sigma.device
        if out is None:
            F = torch.empty((self.P, self.V, C, self.H, self.W), dtype=torch.float32, device=dev)
            A = torch.empty((self.P, self.V, self.H, self.W), dtype=torch.float32, device=dev)
            T = torch.empty_like(A) if want_tfinal else None
            D = torch.empty_like(A)
        else:
            F, A, T, D = out
        self._check(self.lib.art_render_depth(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                              self._flags(fp32_geom, timing), float(depth_sigma), _tptr(F), _tptr(A),
                                              _tptr(T), _tptr(D)),
                    "art_render_depth")
        return F, A, T, D

    def render_sh(self, sigma, feat, lambda_th: float = LAMBDA_TH, fp32_geom: bool = False, timing: bool = False,
                  out=None, want_tfinal: bool = True):
        """Feature maps with view-dependent features (Eq. 2): feat [n][H][C] real
        SH coefficients (H = 1, 4 or 9).  Returns F [P][V][C][H][W], A, T."""
        torch = self._torch
        if feat.dim() != 3:
            raise ValueError("feat must be [n][H][C]")
        H = int(feat.shape[1])
        C, dtype = self._flut(sigma, feat.reshape(feat.shape[0], -1))
        C //= H
        dev = sigma.device
        if out is None:
            F = torch.empty((self.P, self.V, C, self.H, self.W), dtype=torch.float32, device=dev)
            A = torch.empty((self.P, self.V, self.H, self.W), dtype=torch.float32, device=dev)
            T = torch.empty_like(A) if want_tfinal else None
        else:
            F, A, T = out
        self._check(self.lib.art_render_sh(self._h, C, H, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                           self._flags(fp32_geom, timing), _tptr(F), _tptr(A), _tptr(T)),
                    "art_render_sh")
        return F, A, T

    def proposal_labels(self, sigma, feat, lambda_th: float = LAMBDA_TH, fp32_geom: bool = False,
                        timing: bool = False, out=None):
        """Interval labels [P][V][H][W][2] = (u_near, u_far) of every ray from the
        plain traversal ((1, 0) for rays without a composited sample)."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        lab = out if out is not None else torch.empty((self.P, self.V, self.H, self.W, 2), dtype=torch.float32,
                                                      device=sigma.device)
        self._check(self.lib.art_proposal_labels(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                                 self._flags(fp32_geom, timing), _tptr(lab)),
                    "art_proposal_labels")
        return lab

    def render_proposal(self, sigma, feat, intervals, lambda_th: float = LAMBDA_TH,
                        margin_h: float = ART_PROPOSAL_MARGIN_H, f2_tau: float = -1.0, fp32_geom: bool = False,
                        timing: bool = False, out=None, want_tfinal: bool = True, near_only: bool = False):
        """Forward render whose traversal starts from the proposed intervals
        [P][V][H][W][2] (u_near, u_far), with the full traversal as fallback."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        dev = sigma.device
        if out is None:
            F = torch.empty((self.P, self.V, C, self.H, self.W), dtype=torch.float32, device=dev)
            A = torch.empty((self.P, self.V, self.H, self.W), dtype=torch.float32, device=dev)
            T = torch.empty_like(A) if want_tfinal else None
        else:
            F, A, T = out
        iv = None if intervals is None else intervals.contiguous().float()
        flags = self._flags(fp32_geom, timing) | (_lib.ART_PROPOSAL_NEAR_ONLY if near_only else 0)
        self._check(self.lib.art_render_proposal(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                                 flags, _tptr(iv), float(margin_h),
                                                 float(f2_tau), _tptr(F), _tptr(A), _tptr(T)),
                    "art_render_proposal")
        return F, A, T

    # ---- proposal network ----------------------------------------------------------
    def proposal_param_count(self) -> int:
        return int(self.lib.art_proposal_param_count(int(self.J)))

    def set_proposal_weights(self, w) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        self._check(self.lib.art_proposal_set_weights(self._h, w.size, _ptr(w)), "art_proposal_set_weights")

    def init_proposal(self, seed: int) -> None:
        """Seeded initial proposal weights drawn in the library
        (art_proposal_init; resets the Adam state)."""
        self._check(self.lib.art_proposal_init(self._h, int(seed) & ((1 << 64) - 1)), "art_proposal_init")

    def get_proposal_weights(self) -> np.ndarray:
        w = np.zeros(self.proposal_param_count(), dtype=np.float32)
        self._check(self.lib.art_proposal_get_weights(self._h, w.size, _ptr(w)), "art_proposal_get_weights")
        return w

    def proposal_gather(self, ray_id, labels):
        """Network inputs (od [n][6], pose [n]) and targets [n][2] of the rays
        ray_id (int64 indices into [P][V][H][W]) from a label map."""
        torch = self._torch
        ray_id = ray_id.contiguous().to(torch.int64)
        n = ray_id.numel()
        dev = labels.device
        od = torch.empty((n, 6), dtype=torch.float32, device=dev)
        pose = torch.empty((n,), dtype=torch.int32, device=dev)
        tgt = torch.empty((n, 2), dtype=torch.float32, device=dev)
        self._check(self.lib.art_proposal_gather(self._h, n, _tptr(ray_id), _tptr(labels.contiguous()), _tptr(od),
                                                 _tptr(pose), _tptr(tgt)), "art_proposal_gather")
        return od, pose, tgt

    def proposal_forward(self, od, pose):
        torch = self._torch
        out = torch.empty((od.shape[0], 2), dtype=torch.float32, device=od.device)
        self._check(self.lib.art_proposal_forward(self._h, od.shape[0], _tptr(od.contiguous()),
                                                  _tptr(pose.contiguous()), _tptr(out)), "art_proposal_forward")
        return out

    def set_proposal_loss(self, kind: str = "smooth_l1", tau=(0.5, 0.5)) -> None:
        """Training loss of the network: "smooth_l1" or "pinball" at levels
        tau = (tau_near, tau_far) (art_proposal_set_loss)."""
        k = {"smooth_l1": 0, "pinball": 1}[kind]
        self._check(self.lib.art_proposal_set_loss(self._h, k, float(tau[0]), float(tau[1])),
                    "art_proposal_set_loss")

    def proposal_grad(self, od, pose, target):
        """(loss, gradient [count]) of the mean training loss over the rays."""
        torch = self._torch
        g = torch.empty((self.proposal_param_count(),), dtype=torch.float32, device=od.device)
        L = torch.empty((1,), dtype=torch.float32, device=od.device)
        self._check(self.lib.art_proposal_grad(self._h, od.shape[0], _tptr(od.contiguous()),
                                               _tptr(pose.contiguous()), _tptr(target.contiguous()), _tptr(g),
                                               _tptr(L)), "art_proposal_grad")
        return float(L.item()), g

    def calibrate_proposal_margin(self, od, pose, target, quantile: float = 0.999, floor_h: float = 2.0) -> float:
        """Margin (in leaf edges h) that covers the network's late starts on
        held-out rays: the `quantile` of (predicted - true) entry of the first
        sample over the rays that have one, in units of h (at least floor_h);
        computed by the library (art_proposal_calibrate)."""
        m = ctypes.c_float(0.0)
        self._check(self.lib.art_proposal_calibrate(self._h, od.shape[0], _tptr(od.contiguous()),
                                                    _tptr(pose.contiguous()), _tptr(target.contiguous()),
                                                    float(quantile), float(floor_h), ctypes.byref(m)),
                    "art_proposal_calibrate")
        return float(m.value)

    def save_proposal(self, path: str) -> None:
        """Write the network's weights, Adam moments and step count (art_proposal_io)."""
        self._check(self.lib.art_proposal_io(self._h, 1, os.fsencode(path)), "art_proposal_io")

    def load_proposal(self, path: str) -> None:
        """Read a state written by save_proposal; training resumes from it."""
        self._check(self.lib.art_proposal_io(self._h, 0, os.fsencode(path)), "art_proposal_io")

    def proposal_train(self, od, pose, target, batch: int = 16384, steps: int = 1000, lr: float = 1e-3,
                       betas=(0.9, 0.999), eps: float = 1e-8) -> np.ndarray:
        """Adam steps over consecutive batches; returns the batch losses."""
        log = np.zeros(max(steps, 1), dtype=np.float32)
        self._check(self.lib.art_proposal_train(self._h, od.shape[0], _tptr(od.contiguous()),
                                                _tptr(pose.contiguous()), _tptr(target.contiguous()), int(batch),
                                                int(steps), float(lr), float(betas[0]), float(betas[1]), float(eps),
                                                _ptr(log)), "art_proposal_train")
        return log[:steps]

    def backward(self, sigma, feat, F, T, dF, dA=None, lambda_th: float = LAMBDA_TH,
                 fp32_geom: bool = False, timing: bool = False, d_sigma=None, d_feat=None,
                 reuse_build: bool = False, ckpt=None):
        """Accumulate dL/dsigma [n] and dL/dfeat [n][C] (float32) for the last
        render's inputs; returns (d_sigma, d_feat).  reuse_build: use the posed
        octrees and tile lists the last render left when still valid
        (ART_REUSE_BUILD).  ckpt: the checkpoints of render_ckpt (the
        segmented adjoint, art_backward_ckpt)."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        if d_sigma is None:
            d_sigma = torch.zeros((self.n,), dtype=torch.float32, device=sigma.device)
        if d_feat is None:
            d_feat = torch.zeros((self.n, C), dtype=torch.float32, device=sigma.device)
        dF = dF.contiguous().float()
        dA = None if dA is None else dA.contiguous().float()
        flags = self._flags(fp32_geom, timing) | (_lib.ART_REUSE_BUILD if reuse_build else 0)
        if ckpt is not None:
            rec, cnt, K, every = ckpt
            self._check(self.lib.art_backward_ckpt(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                                   flags, _tptr(F), _tptr(T), _tptr(dF), _tptr(dA),
                                                   _tptr(d_sigma), _tptr(d_feat), int(K), int(every), _tptr(rec),
                                                   _tptr(cnt)), "art_backward_ckpt")
            return d_sigma, d_feat
        self._check(self.lib.art_backward(self._h, C, dtype, _tptr(sigma), _tptr(feat), float(lambda_th),
                                          flags, _tptr(F), _tptr(T), _tptr(dF),
                                          _tptr(dA), _tptr(d_sigma), _tptr(d_feat)),
                    "art_backward")
        return d_sigma, d_feat

    # ---- shading network --------------------------------------------------------------
    def shading_param_count(self, C: int) -> int:
        return int(self.lib.art_shading_param_count(int(C)))

    def set_shading_weights(self, C: int, w) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        self._check(self.lib.art_shading_set_weights(self._h, int(C), w.size, _ptr(w)), "art_shading_set_weights")

    def shade(self, F, out=None, no_alloc: bool = False):
        """The Light shading network on feature maps F [N][C][H][W] (float32,
        device; any leading dims are flattened into N): RGB + opacity
        [N][4][H][W].  no_alloc: the library's allocation-free entry point
        (activations in its fixed per-GPU array; batches up to
        ART_SHADING_NOALLOC_BYTES of activations)."""
        torch = self._torch
        C, H, W = int(F.shape[-3]), int(F.shape[-2]), int(F.shape[-1])
        Fc = F.reshape(-1, C, H, W).contiguous().float()
        N = int(Fc.shape[0])
        if out is None:
            out = torch.empty((N, 4, H, W), dtype=torch.float32, device=Fc.device)
        if no_alloc:
            self._check(self.lib.art_shading_forward_noalloc(self._h, C, N, H, W, _tptr(Fc), _tptr(out)),
                        "art_shading_forward_noalloc")
        else:
            self._check(self.lib.art_shading_forward(self._h, C, N, H, W, _tptr(Fc), _tptr(out)),
                        "art_shading_forward")
        return out

    # ---- training step ----------------------------------------------------------------
    def vrt(self, feat, lambda_vrt: float, d_feat=None, fp32_geom: bool = False, reuse_build: bool = False):
        """Voxel regularisation term (Eq. 10) summed over the poses; its gradient
        is added into d_feat [n][C] (float32).  Returns (loss, d_feat).
        reuse_build: use the posed octrees the last render left when still
        valid (ART_REUSE_BUILD)."""
        torch = self._torch
        if feat.dtype not in (torch.float32, torch.bfloat16) or not feat.is_cuda or not feat.is_contiguous():
            raise TypeError("feat must be a contiguous float32 or bfloat16 device tensor")
        if feat.dim() != 2 or feat.shape[0] != self.n:
            raise ValueError(f"expected feat [{self.n}, C]")
        C = int(feat.shape[1])
        dtype = ART_BF16 if feat.dtype == torch.bfloat16 else ART_F32
        if d_feat is None:
            d_feat = torch.zeros((self.n, C), dtype=torch.float32, device=feat.device)
        loss = ctypes.c_double(0.0)
        flags = (ART_GEOM_FP32 if fp32_geom else 0) | (_lib.ART_REUSE_BUILD if reuse_build else 0)
        self._check(self.lib.art_vrt(self._h, C, dtype, _tptr(feat), float(lambda_vrt),
                                     flags, _tptr(d_feat), ctypes.byref(loss)),
                    "art_vrt")
        return float(loss.value), d_feat

    def query(self, pose: int, points, fp32_geom: bool = False):
        """Leaf held by the posed octree of `pose` at each point [n][3] (float64
        device tensor); -1 for empty cells and points outside the root."""
        torch = self._torch
        pts = points.contiguous().to(torch.float64)
        out = torch.empty((pts.shape[0],), dtype=torch.int32, device=pts.device)
        self._check(self.lib.art_query(self._h, int(pose), ART_GEOM_FP32 if fp32_geom else 0, int(pts.shape[0]),
                                       _tptr(pts), _tptr(out)), "art_query")
        return out

    def flut_adam(self, param, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, lower: float = float("-inf")) -> None:
        """In-place Adam update of a float32 FLUT tensor (then param >= lower)."""
        for t in (param, grad, m, v):
            if t.dtype != self._torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != param.numel():
                raise TypeError("param, grad, m, v must be contiguous float32 device tensors of one size")
        self._check(self.lib.art_flut_adam(self._h, int(param.numel()), _tptr(param), _tptr(grad), _tptr(m),
                                           _tptr(v), int(step), float(lr), float(beta1), float(beta2), float(eps),
                                           float(lower)), "art_flut_adam")

    def map_loss(self, F, F_target, A=None, A_target=None):
        """L2 map loss 1/(2R) [sum (F - F*)^2 + sum (A - A*)^2] over the R rays of
        the current poses and cameras (A term when A_target is given) and its
        gradients (art_map_loss): (loss, dL/dF, dL/dA or None)."""
        torch = self._torch
        R = self.P * self.V * self.H * self.W
        F = F.contiguous()
        Ft = F_target.contiguous().float()
        if Ft.shape != F.shape:
            raise ValueError("F_target must have the shape of F")
        dF = torch.empty_like(F)
        dA = None
        At = None
        if A_target is not None:
            A = A.contiguous()
            At = A_target.contiguous().float()
            if At.shape != A.shape or A.numel() != R:
                raise ValueError("A and A_target must hold one value per ray")
            dA = torch.empty_like(A)
        loss = ctypes.c_double(0.0)
        self._check(self.lib.art_map_loss(self._h, F.numel(), R, _tptr(F), _tptr(Ft), _tptr(A) if At is not None else None,
                                          _tptr(At), _tptr(dF), _tptr(dA), ctypes.byref(loss)), "art_map_loss")
        return float(loss.value), dF, dA

    def train_state(self, sigma, feat) -> dict:
        """Adam moments of a float32 FLUT (sigma [n], feat [n][C]) and the step count."""
        torch = self._torch
        return {"step": 0, "m_s": torch.zeros_like(sigma), "v_s": torch.zeros_like(sigma),
                "m_f": torch.zeros_like(feat), "v_f": torch.zeros_like(feat)}

    def train_step(self, sigma, feat, state: dict, F_target, A_target=None, lr: float = 1e-2,
                   lambda_vrt: float = 0.0, lambda_th: float = LAMBDA_TH, fp32_geom: bool = False,
                   segments=None) -> dict:
        """One FLUT training step (Section 3.1, "Training", without the shading
        network): render every pose and view, the map loss
        L_map = 1/(2R) [sum (F - F*)^2 + sum (A - A*)^2] over the R rays (the A
        term when A_target is given), its gradient by the adjoint kernel, the
        voxel regularisation term and its gradient (lambda_vrt > 0), then Adam
        on sigma (projected onto sigma >= 0) and feat, in place.  Returns the
        losses of the FLUT before the update.

        segments = (K, every): the segmented adjoint from ray checkpoints
        (render_ckpt); by default on launches of at most 8M rays (K = 6,
        every = 36: there the adjoint's time is the chain of its longest rays,
        and the checkpoints take (C + 4) x 4 bytes per ray and record), "off"
        to disable."""
        torch = self._torch
        rays = self.P * self.V * self.H * self.W
        if segments is None:
            segments = (6, 36) if rays <= 8 * 1024 * 1024 else "off"
        ck = None

        def render(sync):
            if segments == "off":
                return self.render(sigma, feat, lambda_th, fp32_geom=fp32_geom, sync=sync) + (None,)
            return self.render_ckpt(sigma, feat, lambda_th, K=segments[0], every=segments[1],
                                    fp32_geom=fp32_geom, sync=sync)

        # the render only enqueues its work; the map loss reads its value back
        # (one synchronisation), after which the render's status is read
        # without waiting: a step whose tile lists overflowed renders again
        # with the grown lists (an invalid density raises there)
        F, A, T, ck = render(False)
        l_map, dF, dA = self.map_loss(F, F_target, A, A_target)
        st = self.render_status()
        if st["overflowed_items"] or st["bad_densities"]:
            F, A, T, ck = render(True)
            l_map, dF, dA = self.map_loss(F, F_target, A, A_target)
        # the adjoint and the VRT read the posed octrees (and tile lists) the
        # render just built: the poses and the octree did not change
        d_sigma, d_feat = self.backward(sigma, feat, F, T, dF, dA, lambda_th, fp32_geom=fp32_geom, reuse_build=True,
                                        ckpt=ck)
        l_vrt = 0.0
        if lambda_vrt > 0.0:
            l_vrt, _ = self.vrt(feat, lambda_vrt, d_feat=d_feat, fp32_geom=fp32_geom, reuse_build=True)
        state["step"] += 1
        self.flut_adam(sigma, d_sigma, state["m_s"], state["v_s"], state["step"], lr, lower=0.0)
        self.flut_adam(feat, d_feat, state["m_f"], state["v_f"], state["step"], lr)
        return {"map": l_map, "vrt": l_vrt, "total": l_map + l_vrt}

    # ---- inspection ------------------------------------------------------------------
    def get_bones(self) -> np.ndarray:
        B = np.zeros((self.P, self.J, 3, 4), dtype=np.float64)
        self._check(self.lib.art_get_bones(self._h, _ptr(B)), "art_get_bones")
        return B

    def get_posed_keys(self, pose: int, fp32_geom: bool = False):
        torch = self._torch
        k = torch.empty((self.n,), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(self.lib.art_get_posed_keys(self._h, int(pose), ART_GEOM_FP32 if fp32_geom else 0,
                                                _tptr(k)), "art_get_posed_keys")
        return k.cpu().numpy().view(np.uint32)

    def get_octree(self, pose: int, fp32_geom: bool = False):
        torch = self._torch
        dev = f"cuda:{self.device}"
        counts = np.zeros(4, dtype=np.int64)
        keys = torch.empty((self.n,), dtype=torch.int32, device=dev)
        win = torch.empty_like(keys)
        bk = torch.empty_like(keys)
        br = torch.empty_like(keys)
        bm = torch.empty((self.n, 16), dtype=torch.int32, device=dev)
        self._check(self.lib.art_get_octree(self._h, int(pose), ART_GEOM_FP32 if fp32_geom else 0,
                                            _ptr(counts), _tptr(keys), _tptr(win), _tptr(bk), _tptr(br),
                                            _tptr(bm)), "art_get_octree")
        M, nb = int(counts[0]), int(counts[1])
        u32 = lambda t, m: t[:m].cpu().numpy().view(np.uint32)
        return {"keys": u32(keys, M), "winner": u32(win, M).astype(np.int64),
                "brick_keys": u32(bk, nb), "brick_row": u32(br, nb).astype(np.int64),
                "brick_mask": bm[:nb].cpu().numpy().view(np.uint32),
                "dropped": int(counts[2]), "collisions": int(counts[3])}

    def get_hits(self, pose: int, view: int, sigma, feat, lambda_th: float = 0.0,
                 max_hits: int = 256, fp32_geom: bool = False):
        """Composited samples of every ray of (pose, view): leaf ids [H*W][max_hits],
        chord lengths [H*W][max_hits] (float64), counts [H*W]."""
        torch = self._torch
        C, dtype = self._flut(sigma, feat)
        dev = sigma.device
        HW = self.H * self.W
        leaf = torch.full((HW, max_hits), -1, dtype=torch.int32, device=dev)
        delta = torch.zeros((HW, max_hits), dtype=torch.float64, device=dev)
        count = torch.zeros((HW,), dtype=torch.int32, device=dev)
        self._check(self.lib.art_get_hits(self._h, int(pose), int(view), C, dtype, _tptr(sigma), _tptr(feat),
                                          float(lambda_th), ART_GEOM_FP32 if fp32_geom else 0,
                                          int(max_hits), _tptr(leaf), _tptr(delta), _tptr(count)),
                    "art_get_hits")
        return leaf.cpu().numpy(), delta.cpu().numpy(), count.cpu().numpy()

    def stats(self) -> dict:
        s = np.zeros(_lib.ART_NUM_STATS, dtype=np.int64)
        self._check(self.lib.art_get_stats(self._h, _ptr(s)), "art_get_stats")
        keys = ["rays", "samples", "hit_rays", "dropped", "collisions", "bricks", "pairs", "launches",
                "list_entries", "rounds", "steps", "tile_rays", "proposal_rays", "fallbacks", "grad_adds"]
        return dict(zip(keys, (int(x) for x in s)))

    def timing(self) -> dict:
        ms = np.zeros(7, dtype=np.float32)
        nr = ctypes.c_int(0)
        self._check(self.lib.art_get_timing(self._h, _ptr(ms), ctypes.byref(nr)), "art_get_timing")
        keys = ["fk", "skin", "build", "bin", "render", "total", "proposal"]
        out = dict(zip(keys, (float(x) for x in ms)))
        out["n_render"] = int(nr.value)
        return out


def _make_fn():
    import torch

    class RenderFn(torch.autograd.Function):
        """Differentiable render: (sigma [n], feat [n][C]) -> (F, A).  The
        backward re-traverses every ray in the library's adjoint kernel."""

        @staticmethod
        def forward(ctx, sigma, feat, renderer, lambda_th, fp32_geom):
            F, A, T = renderer.render(sigma.detach(), feat.detach(), lambda_th, fp32_geom)
            ctx.save_for_backward(sigma, feat, F, T)
            ctx.renderer = renderer
            ctx.lambda_th = lambda_th
            ctx.fp32_geom = fp32_geom
            # the adjoint re-traverses the context's current poses and cameras
            ctx.state_version = renderer.state_version()
            return F, A

        @staticmethod
        def backward(ctx, dF, dA):
            sigma, feat, F, T = ctx.saved_tensors
            if ctx.renderer.state_version() != ctx.state_version:
                raise ArtemisError(_lib.ART_ESTATE,
                                   "the octree, skin, skeleton, poses or cameras changed between the forward "
                                   "render and its backward; render again before backward")
            if dF is None:
                dF = torch.zeros_like(F)
            # the octrees of the forward are reused when nothing they depend on changed since
            ds, df = ctx.renderer.backward(sigma.detach(), feat.detach(), F, T, dF, dA,
                                           ctx.lambda_th, ctx.fp32_geom, reuse_build=True)
            return ds.to(sigma.dtype), df.to(feat.dtype), None, None, None

    return RenderFn


RenderFn = None


def render(renderer: Renderer, sigma, feat, lambda_th: float = LAMBDA_TH, fp32_geom: bool = False):
    """Differentiable feature / opacity maps of every pose and camera."""
    global RenderFn
    if RenderFn is None:
        RenderFn = _make_fn()
    return RenderFn.apply(sigma, feat, renderer, lambda_th, fp32_geom)
