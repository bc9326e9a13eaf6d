"""FP64 reference of the FLUT training step: the voxel regularisation term, the
point-query operator Q and the projected Adam update of the FLUT.

TEST INFRASTRUCTURE ONLY (see the package docstring): the plain definitions
the GPU kernels of the training loop are checked against.

Section 3.1 ("Training"): the FLUT is initialised at random and optimised;
under motion several canonical voxels can be warped onto one posed cell, and
the voxel regularisation term (Eq. 10) asks every canonical voxel's feature to
agree with what the posed octree returns at its posed position:

    L_vrt = lambda_vrt / N_v * sum_i || Q(p_i^t, T^t) - f_i^c ||_1

Readings (the paper does not state them):
* Q(p, T^t) is the feature of the voxel the posed octree holds at the posed
  cell containing p, i.e. of that cell's collision winner (the smallest
  canonical leaf id mapped onto it, as in the renderer).  For a winner the
  term is 0.
* The sum and N_v run over the leaves whose posed centre lies inside the posed
  root; a leaf dropped outside the root has no Q.
* Q reads the FLUT, so the gradient reaches both the leaf's own feature and
  the winner's; the subgradient of |x| at 0 is 0.
* The term regularises the features only (not the densities).
* Over a batch of poses the terms of the poses add up.
* The FLUT is updated by Adam; densities are then clamped at 0 (a projection
  keeping every alpha in [0, 1)).
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import INVALID_KEY


def cell_winners(keys: np.ndarray) -> Dict[int, int]:
    """Collision winner (smallest leaf id) of every occupied posed cell, from the
    per-leaf posed keys (INVALID_KEY for dropped leaves), one leaf at a time."""
    win: Dict[int, int] = {}
    for leaf, k in enumerate(np.asarray(keys, dtype=np.int64).tolist()):
        if k == INVALID_KEY:
            continue
        if k not in win or leaf < win[k]:
            win[k] = leaf
    return win


def vrt(keys: np.ndarray, feat: np.ndarray, lambda_vrt: float):
    """L_vrt of one pose (Eq. 10) and its gradient with respect to the features.

    keys: per-leaf posed keys [N]; feat: [N][C] FLUT features.
    Returns (loss, grad [N][C], n_v)."""
    keys = np.asarray(keys, dtype=np.int64)
    feat = np.asarray(feat, dtype=np.float64)
    win = cell_winners(keys)
    inside = keys != INVALID_KEY
    n_v = int(inside.sum())
    grad = np.zeros_like(feat)
    if n_v == 0:
        return 0.0, grad, 0
    scale = lambda_vrt / n_v
    loss = 0.0
    for i in np.nonzero(inside)[0].tolist():
        w = win[int(keys[i])]
        diff = feat[w] - feat[i]            # Q(p_i^t, T^t) - f_i^c
        loss += float(np.abs(diff).sum())
        s = np.sign(diff)
        grad[w] += scale * s
        grad[i] -= scale * s
    return scale * loss, grad, n_v


def query(points: np.ndarray, depth: int, keys: np.ndarray) -> np.ndarray:
    """Q as an index: for every point of the posed space, the canonical leaf the
    posed octree holds at the point's cell (its collision winner), -1 when the
    cell is empty or the point lies outside the posed root [-1, 1)^3.
    keys: per-leaf posed keys of the pose (INVALID_KEY for dropped leaves)."""
    from . import morton30
    win = cell_winners(keys)
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    out = np.full(len(points), -1, dtype=np.int64)
    for n, p in enumerate(np.asarray(points, dtype=np.float64)):
        c = np.floor((p + 1.0) / h).astype(np.int64)
        if np.any(c < 0) or np.any(c >= G):
            continue
        k = int(morton30(c[None, :])[0])
        out[n] = win.get(k, -1)
    return out


def flut_adam(param: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, step: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, lower=None):
    """One Adam update of a FLUT array (step counts from 1), then the optional
    projection onto [lower, inf).  Returns (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    param = param - lr * m_hat / (np.sqrt(v_hat) + eps)
    if lower is not None:
        param = np.maximum(param, lower)
    return param, m, v
