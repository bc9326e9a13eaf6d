"""FP64 CPU oracle of the animated-octree feature renderer.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
definition that the HIP renderer is checked against.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
library never does, and this package imports nothing from the product.

Each function names the passage of the paper it follows (Luo et al., "Artemis:
Articulated Neural Pets with Appearance and Motion Synthesis", 2022):

* ``rodrigues``, ``fk``      - skeleton S = {r, R, T} and the bone transforms
                               M^t_j (M^c_j)^-1 of Eq. 4 (Section 3.1, "Rigging
                               and Deformation"), in FP64;
* ``lbs``                    - linear blend skinning of the leaf centres, Eq. 4;
* ``posed_cells``/``posed_keys`` - the posed voxel of each leaf on the fixed
                               posed lattice (the octree is rebuilt under the
                               pose, Section 3.1, "Dynamic Volume Rendering");
* ``posed_octree``           - occupied cells, the collision winner of each
                               (voxels warped onto one grid cell overwrite each
                               other, Section 3.1 "Training"; the minimum leaf id
                               wins), and the 8^3-brick level of the octree;
* ``camera_rays``            - one ray per pixel r_p = (o_p, d_p);
* ``render``/``backward``    - Eq. 5 and Eq. 6 over the exact ray/voxel chords,
                               the coarse opacity map and the early stop at
                               lambda_th (C code in ``ray_oracle.c``);
* ``render_sh``/``sh_basis`` - Eq. 5 with the view-dependent features of Eq. 2
                               (real SH up to degree 2) at the canonical ray
                               direction d^c = (R_i^t)^-1 d;
* ``mlp``                    - FP64 reference of the ray-interval proposal MLP
                               (not in the paper);
* ``train``                  - the FLUT training step: the voxel regularisation
                               term (Eq. 10), the point-query operator Q and the
                               projected Adam update.

Readings of the paper where it is silent or inconsistent (exclusive
transmittance, chord-length samples, the strict stop test, min-id collision
winner, posed lattice placement, OpenCV cameras) are stated where they are used.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libray_oracle.so")
_lib = None

INVALID_KEY = 0xFFFFFFFF


# ----------------------------------------------------------------------------
# build / load the C part
# ----------------------------------------------------------------------------

def build(force: bool = True) -> str:
    """Compile ray_oracle.c with gcc (FP64, OpenMP)."""
    src = os.path.join(_HERE, "ray_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.oracle_render.restype = ctypes.c_int
    lib.oracle_render.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int64, P, P, ctypes.c_int, P, P, ctypes.c_double,
                                  P, P, P, P, P, P, P, ctypes.c_int, P, P, P, ctypes.c_double, P, ctypes.c_int]
    lib.oracle_backward.restype = ctypes.c_int
    lib.oracle_backward.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int64, P, P, ctypes.c_int, P, P, ctypes.c_double,
                                    P, P, P, P, ctypes.c_int]
    lib.oracle_render_sh.restype = ctypes.c_int
    lib.oracle_render_sh.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int, P, P, P, P,
                                     ctypes.c_double, P, P, P, P, P, ctypes.c_int]
    lib.oracle_sh_basis.restype = None
    lib.oracle_sh_basis.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# skeleton: FK (Eq. 4 bone transforms), FP64
# ----------------------------------------------------------------------------

def rodrigues(r: np.ndarray) -> np.ndarray:
    """Rotation matrix of an axis-angle vector (the joint rotations r of S = {r, R, T}).

    R = I + sin(t) K + (1 - cos(t)) K^2 with t = |r|, K the cross-product matrix
    of r/t; the identity for t < 1e-12."""
    r = np.asarray(r, dtype=np.float64)
    t = math.sqrt(float(r @ r))
    if t < 1e-12:
        return np.eye(3)
    k = r / t
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(t) * K + (1.0 - math.cos(t)) * (K @ K)


def fk(parent: np.ndarray, rest_joint: np.ndarray, r: np.ndarray, R: np.ndarray,
       T: np.ndarray) -> np.ndarray:
    """Skinning matrices B_j = M^t_j (M^c_j)^-1 for every pose (Eq. 4).

    The rest transform of joint j is M^c_j = [I | J_j] (identity rest
    rotations).  The posed transform is the chain
        G_0 = [Rot(R) Rot(r_0) | J_0 + T],
        G_j = G_parent(j) [Rot(r_j) | J_j - J_parent(j)],
    so B_j = G_j [I | -J_j].  Returns float64 [P][J][3][4]."""
    parent = np.asarray(parent)
    Jn = len(parent)
    r = np.asarray(r, dtype=np.float64).reshape(-1, Jn, 3)
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    T = np.asarray(T, dtype=np.float64).reshape(-1, 3)
    rest = np.asarray(rest_joint, dtype=np.float64)
    P = r.shape[0]
    out = np.zeros((P, Jn, 3, 4))
    for p in range(P):
        G = [None] * Jn
        for j in range(Jn):
            L = np.eye(4)
            if parent[j] < 0:
                L[:3, :3] = rodrigues(R[p]) @ rodrigues(r[p, j])
                L[:3, 3] = rest[j] + T[p]
                G[j] = L
            else:
                L[:3, :3] = rodrigues(r[p, j])
                L[:3, 3] = rest[j] - rest[parent[j]]
                G[j] = G[parent[j]] @ L
            inv_rest = np.eye(4)
            inv_rest[:3, 3] = -rest[j]
            out[p, j] = (G[j] @ inv_rest)[:3, :]
    return out


# ----------------------------------------------------------------------------
# skinning and posed cells
# ----------------------------------------------------------------------------

def canonical_centres(ijk: np.ndarray, depth: int) -> np.ndarray:
    """Leaf centres p^c = -1/2 + (ijk + 1/2) h, h = 2^-depth, float64 [N][3]."""
    h = 1.0 / (1 << depth)
    return -0.5 + (np.asarray(ijk, dtype=np.float64).T + 0.5) * h


def lbs(ijk: np.ndarray, depth: int, bone: np.ndarray, weight: np.ndarray,
        B: np.ndarray) -> np.ndarray:
    """Posed leaf centres p^t = sum_k w_k B_{b_k} [p^c; 1] (Eq. 4), float64 [N][3].

    The weights are used as given (no renormalisation); the matrices are blended
    first and then applied, as Eq. 4 is written."""
    pc = canonical_centres(ijk, depth)
    bone = np.asarray(bone).astype(np.int64)          # [4][N]
    w = np.asarray(weight, dtype=np.float64)          # [4][N]
    A = np.zeros((pc.shape[0], 3, 4))
    for k in range(bone.shape[0]):
        A += w[k][:, None, None] * B[bone[k]]
    return np.einsum("nij,nj->ni", A[:, :, :3], pc) + A[:, :, 3]


def posed_cells(pt: np.ndarray, depth: int):
    """Cell of each posed centre on the posed lattice: [-1,1]^3 split into
    G = 2^(depth+1) cells per axis of the canonical leaf size h.

    c = floor((p + 1) / h); a leaf whose cell leaves [0, G)^3 is dropped.
    Returns (cells int64 [N][3], valid bool [N])."""
    h = 1.0 / (1 << depth)
    G = 1 << (depth + 1)
    c = np.floor((pt + 1.0) / h).astype(np.int64)
    valid = np.all((c >= 0) & (c < G), axis=1)
    return c, valid


def morton30(c: np.ndarray) -> np.ndarray:
    """Interleave 10-bit x, y, z cell coordinates into a Morton key (x lowest bit)."""
    c = np.asarray(c, dtype=np.int64)
    key = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(10):
        for a in range(3):
            key |= ((c[:, a] >> b) & 1) << (3 * b + a)
    return key


def posed_keys(cells: np.ndarray, valid: np.ndarray) -> np.ndarray:
    """uint32 Morton key per leaf, INVALID_KEY for dropped leaves."""
    key = np.full(cells.shape[0], INVALID_KEY, dtype=np.int64)
    key[valid] = morton30(cells[valid])
    return key.astype(np.uint32)


def posed_octree(keys: np.ndarray) -> Dict[str, np.ndarray]:
    """Posed octree from per-leaf keys (rebuilt for every pose, Section 3.1).

    * ``keys``/``winner``: the occupied cells in Morton order and, for each, the
      minimum canonical leaf id mapped onto it (collision winner);
    * ``brick_keys``: occupied nodes of the 8^3-leaf level (key >> 9);
    * ``brick_mask``: uint32 [nb][16], bit (key & 511) of each occupied leaf;
    * ``brick_row``: index into ``keys`` of the first leaf of each brick.
    Written with Python dictionaries and sets, one leaf at a time."""
    keys = np.asarray(keys, dtype=np.int64)
    first: Dict[int, int] = {}
    for leaf, k in enumerate(keys.tolist()):
        if k == INVALID_KEY:
            continue
        if k not in first or leaf < first[k]:
            first[k] = leaf
    occ = sorted(first)
    winner = [first[k] for k in occ]
    bricks = sorted({k >> 9 for k in occ})
    bidx = {b: i for i, b in enumerate(bricks)}
    mask = np.zeros((len(bricks), 16), dtype=np.uint32)
    row = np.full(len(bricks), -1, dtype=np.int64)
    for m, k in enumerate(occ):
        b = bidx[k >> 9]
        local = k & 511
        mask[b, local >> 5] |= np.uint32(1 << (local & 31))
        if row[b] < 0:
            row[b] = m
    return {
        "keys": np.array(occ, dtype=np.uint32),
        "winner": np.array(winner, dtype=np.int64),
        "brick_keys": np.array(bricks, dtype=np.uint32),
        "brick_mask": mask,
        "brick_row": row,
        "dropped": int(np.sum(keys == INVALID_KEY)),
    }


def occupancy_from_cells(cells: np.ndarray, valid: np.ndarray, depth: int):
    """Sorted linear cell keys (cz*G + cy)*G + cx of the occupied posed cells and
    the min-id winner leaf of each (for the ray oracle)."""
    G = 1 << (depth + 1)
    leaf = np.nonzero(valid)[0]
    c = cells[valid]
    lin = (c[:, 2] * G + c[:, 1]) * G + c[:, 0]
    order = np.lexsort((leaf, lin))          # by key, then by leaf id
    lin = lin[order]
    leaf = leaf[order]
    first = np.ones(len(lin), dtype=bool)
    first[1:] = lin[1:] != lin[:-1]
    return np.ascontiguousarray(lin[first]), np.ascontiguousarray(leaf[first])


def canonical_occupancy(ijk: np.ndarray, depth: int):
    """Occupancy of the un-warped canonical octree placed on the posed lattice
    (canonical cell + 2^(depth-1) on each axis, the same leaf size)."""
    c = np.asarray(ijk, dtype=np.int64).T + (1 << (depth - 1))
    return occupancy_from_cells(c, np.ones(c.shape[0], dtype=bool), depth)


# ----------------------------------------------------------------------------
# cameras and rays
# ----------------------------------------------------------------------------

def camera_rays(K: np.ndarray, c2w: np.ndarray, H: int, W: int):
    """One ray per pixel of an OpenCV pinhole camera (pixel centres at +1/2).

    d_cam = ((x + 1/2 - cx)/fx, (y + 1/2 - cy)/fy, 1), d = normalize(R d_cam),
    o = camera centre.  Returns o, d as float64 [V][H][W][3]."""
    K = np.asarray(K, dtype=np.float64).reshape(-1, 3, 3)
    c2w = np.asarray(c2w, dtype=np.float64).reshape(-1, 3, 4)
    V = K.shape[0]
    o = np.zeros((V, H, W, 3))
    d = np.zeros((V, H, W, 3))
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    for v in range(V):
        fx, fy, cx, cy = K[v, 0, 0], K[v, 1, 1], K[v, 0, 2], K[v, 1, 2]
        dc = np.stack([(xs + 0.5 - cx) / fx, (ys + 0.5 - cy) / fy, np.ones_like(xs)], axis=-1)
        dw = dc @ c2w[v, :, :3].T
        d[v] = dw / np.linalg.norm(dw, axis=-1, keepdims=True)
        o[v] = c2w[v, :, 3]
    return o, d


# ----------------------------------------------------------------------------
# rendering (C, FP64)
# ----------------------------------------------------------------------------

def render(o: np.ndarray, d: np.ndarray, depth: int, occ_key: np.ndarray, occ_leaf: np.ndarray,
           sigma: np.ndarray, feat: np.ndarray, lambda_th: float, max_hits: int = 0,
           n_threads: int = 0, depth_sigma: float = 0.0) -> Dict[str, np.ndarray]:
    """Eq. 5-6 per ray over the exact voxel chords (see ray_oracle.c).

    o, d: [n][3] float64 rays (|d| = 1).  Returns F [n][C], A [n], T [n],
    n_comp [n], n_hit [n], min_gap [n], min_tgap [n] and, when max_hits > 0,
    hit_leaf/hit_delta [n][max_hits] of the composited samples, and seg [n][4]:
    t_a, t_b of the clipped ray (NaN on a miss) and the entry t of the first /
    exit t of the last composited sample (NaN without samples), and dist [n]:
    the entry t of the first occupied voxel along the whole clipped ray with
    density > depth_sigma, whether or not the early stop came before it (+inf
    without one) - the depth buffer of the hybrid rendering (Section 3.1,
    paragraph "Hybrid Rendering")."""
    lib = _load()
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    C = feat.shape[1]
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    occ_key = np.ascontiguousarray(occ_key, dtype=np.int64)
    occ_leaf = np.ascontiguousarray(occ_leaf, dtype=np.int64)
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    out = {
        "F": np.zeros((n, C)), "A": np.zeros(n), "T": np.ones(n),
        "n_comp": np.zeros(n, dtype=np.int32), "n_hit": np.zeros(n, dtype=np.int32),
        "min_gap": np.zeros(n), "min_tgap": np.zeros(n), "seg": np.zeros((n, 4)), "dist": np.zeros(n),
    }
    hl = hd = None
    if max_hits > 0:
        hl = np.full((n, max_hits), -1, dtype=np.int64)
        hd = np.zeros((n, max_hits))
        out["hit_leaf"], out["hit_delta"] = hl, hd
    rc = lib.oracle_render(n, _ptr(o), _ptr(d), G, h, len(occ_key), _ptr(occ_key), _ptr(occ_leaf),
                           C, _ptr(sigma), _ptr(feat), float(lambda_th),
                           _ptr(out["F"]), _ptr(out["A"]), _ptr(out["T"]), _ptr(out["n_comp"]),
                           _ptr(out["n_hit"]), _ptr(out["min_gap"]), _ptr(out["min_tgap"]),
                           int(max_hits), _ptr(hl), _ptr(hd), _ptr(out["seg"]), float(depth_sigma),
                           _ptr(out["dist"]), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle_render failed")
    return out


def sh_basis(H: int, dirs: np.ndarray) -> np.ndarray:
    """Real SH basis values Y_0..Y_{H-1} (Eq. 2; H = 1, 4, 9) at unit directions
    [n][3], from ray_oracle.c."""
    lib = _load()
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], 9))
    for i, (x, y, z) in enumerate(dirs.tolist()):
        lib.oracle_sh_basis(int(H), x, y, z, _ptr(out[i]))
    return out[:, :H]


def dominant_bone(bone: np.ndarray, weight: np.ndarray) -> np.ndarray:
    """Per leaf, the bone of its largest skin weight (the first of equal ones):
    the bone whose rotation stands for the voxel rotation R_i^t."""
    bone = np.asarray(bone)
    weight = np.asarray(weight)
    slot = np.argmax(weight, axis=0)
    return bone[slot, np.arange(bone.shape[1])].astype(np.int32)


def render_sh(o: np.ndarray, d: np.ndarray, depth: int, occ_key: np.ndarray, occ_leaf: np.ndarray,
              sigma: np.ndarray, feat: np.ndarray, H: int, dom_bone: np.ndarray, B_pose: np.ndarray,
              lambda_th: float, n_threads: int = 0):
    """Eq. 5 with the view-dependent feature S(f, d^c) of Eq. 2: feat [N][H][C]
    SH coefficients, d^c = R^T d with R the rotation of the leaf's dominant bone
    in the pose (B_pose [J][3][4]).  Returns F [n][C], A, T and the guard-band
    measures min_gap, min_tgap."""
    lib = _load()
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    N = feat.shape[0]
    C = feat.shape[-1]
    assert feat.shape == (N, H, C)
    rot = np.ascontiguousarray(np.asarray(B_pose, dtype=np.float64)[:, :, :3].reshape(-1, 9))
    out = {"F": np.zeros((n, C)), "A": np.zeros(n), "T": np.zeros(n), "min_gap": np.zeros(n),
           "min_tgap": np.zeros(n)}
    rc = lib.oracle_render_sh(n, _ptr(o), _ptr(d), 1 << (depth + 1), 1.0 / (1 << depth), len(occ_key),
                              _ptr(np.ascontiguousarray(occ_key, dtype=np.int64)),
                              _ptr(np.ascontiguousarray(occ_leaf, dtype=np.int64)), C, H,
                              _ptr(np.ascontiguousarray(sigma, dtype=np.float64)), _ptr(feat),
                              _ptr(np.ascontiguousarray(dom_bone, dtype=np.int32)), _ptr(rot), float(lambda_th),
                              _ptr(out["F"]), _ptr(out["A"]), _ptr(out["T"]), _ptr(out["min_gap"]),
                              _ptr(out["min_tgap"]), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle_render_sh failed")
    return out


def interval_labels(seg: np.ndarray) -> np.ndarray:
    """Training labels of the ray-interval proposal from ``render(...)["seg"]``:
    u_near / u_far = entry t of the first / exit t of the last composited sample,
    mapped to [0, 1] over the ray's span [t_a, t_b] inside the posed root.  A ray
    with no composited sample (including one that misses the root) gets the
    empty interval (1, 0)."""
    seg = np.asarray(seg, dtype=np.float64).reshape(-1, 4)
    out = np.empty((seg.shape[0], 2))
    out[:, 0] = 1.0
    out[:, 1] = 0.0
    hit = np.isfinite(seg[:, 2])
    span = seg[hit, 1] - seg[hit, 0]
    out[hit, 0] = (seg[hit, 2] - seg[hit, 0]) / span
    out[hit, 1] = (seg[hit, 3] - seg[hit, 0]) / span
    return out


def backward(o: np.ndarray, d: np.ndarray, depth: int, occ_key: np.ndarray, occ_leaf: np.ndarray,
             sigma: np.ndarray, feat: np.ndarray, lambda_th: float, gF: np.ndarray,
             gA: Optional[np.ndarray] = None, n_threads: int = 0):
    """Gradients of a loss with dL/dF = gF [n][C], dL/dA = gA [n] with respect to
    the leaf densities [N] and features [N][C] (FP64, explicit suffix sums)."""
    lib = _load()
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    N, C = feat.shape
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    gF = np.ascontiguousarray(gF, dtype=np.float64).reshape(n, C)
    gA = None if gA is None else np.ascontiguousarray(gA, dtype=np.float64).reshape(n)
    occ_key = np.ascontiguousarray(occ_key, dtype=np.int64)
    occ_leaf = np.ascontiguousarray(occ_leaf, dtype=np.int64)
    dsig = np.zeros(N)
    dfeat = np.zeros((N, C))
    rc = lib.oracle_backward(n, _ptr(o), _ptr(d), 1 << (depth + 1), 1.0 / (1 << depth),
                             len(occ_key), _ptr(occ_key), _ptr(occ_leaf), C, _ptr(sigma),
                             _ptr(feat), float(lambda_th), _ptr(gF), _ptr(gA), _ptr(dsig),
                             _ptr(dfeat), int(n_threads))
    if rc != 0:
        raise MemoryError("oracle_backward failed")
    return dsig, dfeat


# ----------------------------------------------------------------------------
# whole-pipeline convenience
# ----------------------------------------------------------------------------

def pose_occupancy(ijk, depth, bone, weight, B_pose):
    """(occ_key, occ_leaf, cells, valid, p^t) of one pose."""
    pt = lbs(ijk, depth, bone, weight, B_pose)
    cells, valid = posed_cells(pt, depth)
    occ_key, occ_leaf = occupancy_from_cells(cells, valid, depth)
    return occ_key, occ_leaf, cells, valid, pt


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even), returned
    as float32 - the storage rounding of the BF16 leaf form."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), x, out)


def map_rel_error(F: np.ndarray, F_ref: np.ndarray):
    """Per-map error norms: rel_max = max|F - F_ref| / max|F_ref| and
    rel_mean = sum|F - F_ref| / sum|F_ref| (0 when the reference map is zero)."""
    F = np.asarray(F, dtype=np.float64)
    R = np.asarray(F_ref, dtype=np.float64)
    den_max = np.abs(R).max()
    den_sum = np.abs(R).sum()
    diff = np.abs(F - R)
    rmax = float(diff.max() / den_max) if den_max > 0 else float(diff.max())
    rmean = float(diff.sum() / den_sum) if den_sum > 0 else float(diff.sum())
    return rmax, rmean
