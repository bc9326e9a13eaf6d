"""Seeded synthetic inputs for the animated-octree feature renderer.

This module only *draws data*: animal-shaped canonical octrees (a voxelised
union of jittered ellipsoids), a skeleton inside them, per-leaf skin weights,
random poses, ring cameras, target maps and random training-ray draws.  It holds
none of the renderer's arithmetic (no skinning, no octree build, no ray
traversal, no compositing), so both the FP64 oracle and the HIP path can take
their inputs from here without sharing any code of the method.

The paper's own inputs (CGI animals carved from multi-view alpha mattes, skin
weights blended from a skinned mesh, captured motion) are not available; these
stand in for them:

* leaves: cells of a 2^D canonical grid over [-1/2, 1/2]^3 whose centre lies in
  the ellipsoid union; a global scale is bisected until the leaf count is within
  2% of the target (Section 3.1, "Octree Feature Indexing" carves a voxel array
  P; here a union of ellipsoids replaces the carved hull);
* skin weights: normalised inverse distance to the 4 nearest bone segments,
  w_k ~ 1/max(d_k, h/2), ties to the lower bone id (replaces the mesh-based
  blend of Eq. 3, which needs a skinned mesh);
* poses: per-bone axis-angle with a uniform random axis and angle in
  [-30 deg, 30 deg] (the skeleton parameter S = {r, R, T} of Section 3.1,
  "Rigging and Deformation"); global R = T = 0;
* cameras: OpenCV pinhole cameras on a ring around the animal.

Leaves are listed in canonical Morton order (x in the lowest bit), the natural
order of an octree's leaf array.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "SceneConfig", "Scene", "CONFIGS", "make_scene", "make_poses", "make_cameras", "make_shading_weights",
    "shading_shapes",
    "make_targets", "sample_training_rays", "rotation_about",
]


# ----------------------------------------------------------------------------
# configurations (the five workloads)
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class SceneConfig:
    name: str
    depth: int                 # canonical octree depth D (grid 2^D per axis)
    n_target: int              # target number of occupied leaves
    layout: str                # "small" (8 ellipsoids, 12 bones) or "full" (24, 40)
    C: int                     # feature channels
    sigma_dist: str            # "uniform5_50" or "loguniform1_100"
    n_poses: int
    n_views: int
    height: int
    width: int
    storage: str = "f32"       # "f32" or "bf16"
    geom_seed: int = 1
    appearance_seed: int = 2
    target_seed: int = 3
    mlp_seed: int = 4
    ray_seed: int = 5
    pose_seed0: int = 1000


CONFIGS: Dict[str, SceneConfig] = {
    # plain renderer, tiny
    "tiny": SceneConfig("tiny", 6, 20_000, "small", 8, "uniform5_50", 1, 1, 128, 128),
    # plain renderer, full size, FP32
    "full": SceneConfig("full", 9, 1_500_000, "full", 16, "loguniform1_100", 30, 8, 512, 512),
    # precision form: BF16 storage, 16 cameras at 1024^2 (30 poses as the full scene)
    "bf16": SceneConfig("bf16", 9, 1_500_000, "full", 16, "loguniform1_100", 30, 16, 1024, 1024,
                        storage="bf16"),
    # differentiation form: 4 cameras at 512^2, one pose
    "grad": SceneConfig("grad", 9, 1_500_000, "full", 16, "loguniform1_100", 1, 4, 512, 512),
    # learned-proposal form: 16 cameras at 1024^2, 60 poses
    "proposal": SceneConfig("proposal", 9, 1_500_000, "full", 16, "loguniform1_100", 60, 16,
                            1024, 1024),
}


# ----------------------------------------------------------------------------
# small geometry helpers (data generation only)
# ----------------------------------------------------------------------------

def rotation_about(axis: np.ndarray, angle: float) -> np.ndarray:
    """3x3 rotation by `angle` about unit `axis` (used only to orient ellipsoids)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    x, y, z = a
    c, s = math.cos(angle), math.sin(angle)
    C = 1.0 - c
    return np.array([
        [c + x * x * C, x * y * C - z * s, x * z * C + y * s],
        [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
        [z * x * C - y * s, z * y * C + x * s, c + z * z * C],
    ])


def _pitch(deg: float) -> Tuple[float, float, float, float]:
    # rotation about +y: positive tilts +x towards -z
    return (0.0, 1.0, 0.0, math.radians(deg))


# An ellipsoid template entry: (centre xyz, semi-axes xyz, (axis xyz, angle) or None)
_Ell = Tuple[Tuple[float, float, float], Tuple[float, float, float], Optional[Tuple[float, float, float, float]]]


def _layout_small() -> Tuple[List[_Ell], np.ndarray, np.ndarray, List[str]]:
    """8 ellipsoids (body, neck, head, tail, 4 legs) and a 12-bone tree."""
    ells: List[_Ell] = [
        ((0.00, 0.00, 0.02), (0.36, 0.30, 0.26), None),                  # body
        ((0.33, 0.00, 0.16), (0.13, 0.10, 0.10), _pitch(-40)),           # neck
        ((0.43, 0.00, 0.27), (0.14, 0.13, 0.13), None),                  # head
        ((-0.36, 0.00, 0.16), (0.13, 0.055, 0.055), _pitch(45)),         # tail
        ((0.20, 0.12, -0.24), (0.11, 0.11, 0.15), None),                 # leg FL
        ((0.20, -0.12, -0.24), (0.11, 0.11, 0.15), None),                # leg FR
        ((-0.20, 0.12, -0.24), (0.11, 0.11, 0.15), None),                # leg HL
        ((-0.20, -0.12, -0.24), (0.11, 0.11, 0.15), None),             # leg HR
    ]
    names = ["root", "spine", "chest", "neck", "head", "tail1", "tail2", "tail3",
             "legFL", "legFR", "legHL", "legHR"]
    joints = np.array([
        [0.00, 0.00, 0.00],   # root (body centre)
        [0.12, 0.00, 0.03],   # spine
        [0.24, 0.00, 0.06],   # chest
        [0.32, 0.00, 0.14],   # neck
        [0.42, 0.00, 0.25],   # head
        [-0.28, 0.00, 0.08],  # tail1
        [-0.35, 0.00, 0.15],  # tail2
        [-0.42, 0.00, 0.22],  # tail3
        [0.20, 0.12, -0.10],  # leg FL
        [0.20, -0.12, -0.10],  # leg FR
        [-0.20, 0.12, -0.10],  # leg HL
        [-0.20, -0.12, -0.10],  # leg HR
    ])
    parent = np.array([-1, 0, 1, 2, 3, 0, 5, 6, 2, 2, 0, 0], dtype=np.int32)
    return ells, joints, parent, names


def _layout_full() -> Tuple[List[_Ell], np.ndarray, np.ndarray, List[str]]:
    """24 ellipsoids and a 40-bone quadruped tree."""
    ells: List[_Ell] = [
        ((-0.18, 0.00, 0.02), (0.17, 0.12, 0.12), None),                 # rump
        ((0.02, 0.00, 0.00), (0.17, 0.11, 0.11), None),                  # belly
        ((0.22, 0.00, 0.03), (0.15, 0.12, 0.13), None),                  # chest
        ((0.38, 0.00, 0.11), (0.075, 0.065, 0.065), _pitch(-45)),        # neck 1
        ((0.44, 0.00, 0.19), (0.065, 0.06, 0.06), _pitch(-50)),          # neck 2
        ((0.51, 0.00, 0.25), (0.075, 0.065, 0.065), None),               # cranium
        ((0.59, 0.00, 0.22), (0.065, 0.04, 0.04), None),                 # snout
        ((0.50, 0.045, 0.33), (0.022, 0.016, 0.045), None),              # ear L
        ((0.50, -0.045, 0.33), (0.022, 0.016, 0.045), None),             # ear R
        ((-0.38, 0.00, 0.05), (0.065, 0.028, 0.028), _pitch(13)),        # tail 1
        ((-0.48, 0.00, 0.07), (0.065, 0.026, 0.026), _pitch(13)),        # tail 2
        ((-0.58, 0.00, 0.09), (0.065, 0.024, 0.024), _pitch(13)),        # tail 3
    ]
    for x, y in ((0.26, 0.09), (0.26, -0.09), (-0.22, 0.09), (-0.22, -0.09)):
        ells.append(((x, y, -0.12), (0.045, 0.045, 0.085), None))        # upper leg
        ells.append(((x + 0.01, y, -0.28), (0.034, 0.034, 0.075), None))  # lower leg
    for x, y in ((0.26, 0.09), (0.26, -0.09), (-0.22, 0.09), (-0.22, -0.09)):
        ells.append(((x + 0.03, y, -0.37), (0.05, 0.034, 0.022), None))   # paw
    names = ["root", "spine1", "spine2", "spine3", "chest", "neck1", "neck2", "head", "jaw",
             "earL", "earR"] + [f"tail{k + 1}" for k in range(9)]
    joints = [
        [0.00, 0.00, 0.00],
        [0.07, 0.00, 0.01],
        [0.14, 0.00, 0.02],
        [0.21, 0.00, 0.03],
        [0.29, 0.00, 0.04],
        [0.37, 0.00, 0.10],
        [0.43, 0.00, 0.18],
        [0.50, 0.00, 0.24],
        [0.58, 0.00, 0.20],
        [0.50, 0.045, 0.31],
        [0.50, -0.045, 0.31],
    ]
    parent = [-1, 0, 1, 2, 3, 4, 5, 6, 7, 7, 7]
    for k in range(9):
        joints.append([-0.30 - 0.042 * k, 0.0, 0.04 + 0.007 * k])
        parent.append(0 if k == 0 else 10 + k)
    leg_names = ["FL", "FR", "HL", "HR"]
    for li, (x, y) in enumerate(((0.26, 0.09), (0.26, -0.09), (-0.22, 0.09), (-0.22, -0.09))):
        attach = 4 if li < 2 else 0
        base = len(joints)
        pts = [[x, y * 0.9, -0.02], [x, y, -0.12], [x + 0.01, y, -0.24], [x, y, -0.33],
               [x + 0.03, y, -0.37]]
        for k, p in enumerate(pts):
            joints.append(p)
            parent.append(attach if k == 0 else base + k - 1)
            names.append(f"leg{leg_names[li]}{k + 1}")
    return ells, np.array(joints, dtype=np.float64), np.array(parent, dtype=np.int32), names


def _jitter(ells: List[_Ell], joints: np.ndarray, parent: np.ndarray, seed: int):
    """Centres +-10% of the mean bone length, semi-axes x U(0.85,1.15), orientation +-10 deg."""
    rng = np.random.default_rng(seed)
    seg = np.array([np.linalg.norm(joints[j] - joints[parent[j]]) for j in range(1, len(parent))])
    L = float(seg.mean())
    centres, axes, rots = [], [], []
    for c, a, rot in ells:
        c = np.array(c) + rng.uniform(-0.1, 0.1, 3) * L
        a = np.array(a) * rng.uniform(0.85, 1.15, 3)
        R = np.eye(3) if rot is None else rotation_about(np.array(rot[:3]), rot[3])
        ax = rng.normal(size=3)
        R = rotation_about(ax, math.radians(rng.uniform(-10.0, 10.0))) @ R
        centres.append(c)
        axes.append(a)
        rots.append(R)
    return np.array(centres), np.array(axes), np.array(rots)


def _voxelise(centres, axes, rots, scale: float, depth: int) -> np.ndarray:
    """Boolean occupancy of the 2^depth canonical grid: cell centre inside the union."""
    G = 1 << depth
    h = 1.0 / G
    occ = np.zeros((G, G, G), dtype=bool)   # indexed [i, j, k] = [x, y, z]
    for c, a, R in zip(centres, axes, rots):
        c = c * scale
        a = a * scale
        # axis-aligned bounding box of the rotated ellipsoid
        ext = np.sqrt((R ** 2) @ (a ** 2))
        lo = np.floor((c - ext + 0.5) / h - 0.5).astype(int)
        hi = np.ceil((c + ext + 0.5) / h - 0.5).astype(int)
        if np.any(lo < 0) or np.any(hi >= G):
            raise ValueError("ellipsoid leaves the canonical root")
        ii = np.arange(lo[0], hi[0] + 1)
        jj = np.arange(lo[1], hi[1] + 1)
        kk = np.arange(lo[2], hi[2] + 1)
        px = -0.5 + (ii + 0.5) * h - c[0]
        py = -0.5 + (jj + 0.5) * h - c[1]
        pz = -0.5 + (kk + 0.5) * h - c[2]
        # local coordinates u = R^T (p - c), tested as sum (u/a)^2 <= 1
        acc = np.zeros((len(ii), len(jj), len(kk)))
        for r in range(3):
            u = (R[0, r] * px[:, None, None] + R[1, r] * py[None, :, None]
                 + R[2, r] * pz[None, None, :]) / a[r]
            acc += u * u
        occ[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] |= acc <= 1.0
    return occ


def _morton3(i: np.ndarray, j: np.ndarray, k: np.ndarray, bits: int) -> np.ndarray:
    out = np.zeros(i.shape, dtype=np.uint64)
    for b in range(bits):
        out |= ((i.astype(np.uint64) >> b) & 1) << np.uint64(3 * b)
        out |= ((j.astype(np.uint64) >> b) & 1) << np.uint64(3 * b + 1)
        out |= ((k.astype(np.uint64) >> b) & 1) << np.uint64(3 * b + 2)
    return out


def _bone_segments(joints: np.ndarray, parent: np.ndarray):
    """Segment of bone j: from joint j to the mean of its children (tips extend the parent bone)."""
    J = len(parent)
    a = joints.copy()
    b = np.empty_like(joints)
    for j in range(J):
        kids = np.nonzero(parent == j)[0]
        if len(kids):
            b[j] = joints[kids].mean(axis=0)
        elif parent[j] >= 0:
            b[j] = joints[j] + 0.5 * (joints[j] - joints[parent[j]])
        else:
            b[j] = joints[j]
    return a, b


def _skin_weights(p: np.ndarray, joints: np.ndarray, parent: np.ndarray, h: float):
    """4 nearest bone segments, w ~ 1/max(d, h/2), normalised; ties to the lower bone id."""
    a, b = _bone_segments(joints, parent)
    J = len(parent)
    d = np.empty((p.shape[0], J))
    for j in range(J):
        ab = b[j] - a[j]
        L2 = float(ab @ ab)
        ap = p - a[j]
        t = np.zeros(p.shape[0]) if L2 == 0.0 else np.clip(ap @ ab / L2, 0.0, 1.0)
        q = ap - t[:, None] * ab[None, :]
        d[:, j] = np.sqrt(np.einsum("ij,ij->i", q, q))
    order = np.argsort(d, axis=1, kind="stable")[:, :4]
    dk = np.take_along_axis(d, order, axis=1)
    inv = 1.0 / np.maximum(dk, 0.5 * h)
    w = inv / inv.sum(axis=1, keepdims=True)
    return order.astype(np.uint8), w


# ----------------------------------------------------------------------------
# the scene
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    config: SceneConfig
    depth: int
    ijk: np.ndarray          # uint16 [3][N] canonical cells (SoA planes), Morton-ordered
    bone: np.ndarray         # uint8 [4][N] bone ids (SoA planes)
    weight: np.ndarray       # float32 [4][N] skin weights (SoA planes), sum ~ 1
    parent: np.ndarray       # int32 [J]
    rest_joint: np.ndarray   # float64 [J][3] joint positions in the canonical pose
    sigma: np.ndarray        # float32 [N] densities
    feat: np.ndarray         # float32 [N][C] features (leaf-major rows)
    scale: float
    centre: np.ndarray       # float64 [3] bounding-box centre of the canonical leaves
    r_bs: float              # bounding-sphere radius about `centre`

    @property
    def n(self) -> int:
        return int(self.ijk.shape[1])

    @property
    def J(self) -> int:
        return int(self.parent.shape[0])

    @property
    def C(self) -> int:
        return int(self.feat.shape[1])


def _bisect_scale(centres, axes, rots, depth: int, n_target: int) -> Tuple[float, np.ndarray]:
    lo, hi = 0.05, 2.0
    best = None
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        try:
            occ = _voxelise(centres, axes, rots, mid, depth)
        except ValueError:
            hi = mid
            continue
        n = int(occ.sum())
        if abs(n - n_target) <= 0.02 * n_target:
            # tighten towards the target a little more, but accept this one
            best = (mid, occ)
            if abs(n - n_target) <= 0.002 * n_target:
                break
        if n < n_target:
            lo = mid
        else:
            hi = mid
    if best is None:
        raise RuntimeError("could not reach the leaf-count target inside the canonical root")
    return best


@functools.lru_cache(maxsize=8)
def _scene_geometry(layout: str, depth: int, n_target: int, seed: int):
    ells, joints, parent, _names = _layout_small() if layout == "small" else _layout_full()
    centres, axes, rots = _jitter(ells, joints, parent, seed)
    scale, occ = _bisect_scale(centres, axes, rots, depth, n_target)
    i, j, k = np.nonzero(occ)
    order = np.argsort(_morton3(i, j, k, depth), kind="stable")
    ijk = np.stack([i[order], j[order], k[order]]).astype(np.uint16)
    h = 1.0 / (1 << depth)
    p = -0.5 + (ijk.T.astype(np.float64) + 0.5) * h
    rest = joints * scale
    bone, w = _skin_weights(p, rest, parent, h)
    lo = p.min(axis=0) - 0.5 * h
    hi = p.max(axis=0) + 0.5 * h
    centre = 0.5 * (lo + hi)
    r_bs = float(np.sqrt(((p - centre) ** 2).sum(axis=1)).max() + 0.5 * math.sqrt(3) * h)
    return (ijk, np.ascontiguousarray(bone.T), np.ascontiguousarray(w.T.astype(np.float32)),
            parent, rest, scale, centre, r_bs)


def make_scene(cfg: SceneConfig | str, n_target: Optional[int] = None,
               depth: Optional[int] = None, C: Optional[int] = None) -> Scene:
    """Build the seeded scene for a configuration (optionally overriding size knobs)."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if n_target is not None or depth is not None or C is not None:
        cfg = dataclasses.replace(cfg, n_target=n_target or cfg.n_target,
                                  depth=depth or cfg.depth, C=C or cfg.C)
    ijk, bone, w, parent, rest, scale, centre, r_bs = _scene_geometry(
        cfg.layout, cfg.depth, cfg.n_target, cfg.geom_seed)
    N = ijk.shape[1]
    rng = np.random.default_rng(cfg.appearance_seed)
    if cfg.sigma_dist == "uniform5_50":
        sigma = rng.uniform(5.0, 50.0, N)
    else:
        sigma = np.exp(rng.uniform(0.0, math.log(100.0), N))
    feat = rng.normal(size=(N, cfg.C))
    return Scene(cfg, cfg.depth, ijk, bone, w, parent.copy(), rest.copy(),
                 sigma.astype(np.float32), feat.astype(np.float32), scale, centre, r_bs)


def make_poses(J: int, P: int, seed0: int = 1000, max_deg: float = 30.0):
    """Axis-angle per bone (uniform axis, angle ~ U(-max,max)); global R = T = 0.

    Returns r [P][J][3], R [P][3], T [P][3] (float64)."""
    r = np.zeros((P, J, 3))
    for p in range(P):
        rng = np.random.default_rng(seed0 + p)
        ax = rng.normal(size=(J, 3))
        ax /= np.linalg.norm(ax, axis=1, keepdims=True)
        ang = rng.uniform(-math.radians(max_deg), math.radians(max_deg), J)
        r[p] = ax * ang[:, None]
    return r, np.zeros((P, 3)), np.zeros((P, 3))


def make_cameras(scene: Scene, V: int, H: int, W: int, elevation_deg: float = 15.0,
                 azimuth0_deg: float = 7.5, radius_factor: float = 2.5):
    """OpenCV pinhole ring cameras looking at the canonical bbox centre, up = +z.

    Returns K [V][3][3] and cam_to_world [V][3][4] (float64); columns of the
    rotation are the camera x (right), y (down) and z (forward) axes."""
    radius = radius_factor * scene.r_bs
    fy = 0.5 * H * radius / (1.1 * scene.r_bs)       # vertical FOV = 2 atan(1.1 r_bs / radius)
    K = np.zeros((V, 3, 3))
    c2w = np.zeros((V, 3, 4))
    el = math.radians(elevation_deg)
    up = np.array([0.0, 0.0, 1.0])
    for v in range(V):
        az = math.radians(360.0 * v / V + azimuth0_deg)
        pos = scene.centre + radius * np.array([math.cos(el) * math.cos(az),
                                                math.cos(el) * math.sin(az), math.sin(el)])
        fwd = scene.centre - pos
        fwd /= np.linalg.norm(fwd)
        right = np.cross(fwd, up)
        right /= np.linalg.norm(right)
        down = np.cross(fwd, right)
        K[v] = [[fy, 0.0, 0.5 * W], [0.0, fy, 0.5 * H], [0.0, 0.0, 1.0]]
        c2w[v, :, 0] = right
        c2w[v, :, 1] = down
        c2w[v, :, 2] = fwd
        c2w[v, :, 3] = pos
    return K, c2w


def make_targets(P: int, V: int, C: int, H: int, W: int, seed: int = 3) -> np.ndarray:
    """Target feature maps F* ~ N(0,1), shape [P][V][C][H][W] (float32)."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=(P, V, C, H, W)).astype(np.float32)


def make_mlp_init(J: int, seed: int = 4, hidden: int = 64) -> np.ndarray:
    """Initial FP32 parameters of the ray-interval proposal network
    (6 + 6J -> hidden -> hidden -> hidden -> 2), flat in the order W1, b1, W2,
    b2, W3, b3, W4, b4 (weights row-major [out][in]): every weight and bias of a
    layer with fan-in m drawn from U(-1/sqrt(m), 1/sqrt(m))."""
    rng = np.random.default_rng(seed)
    dims = [6 + 6 * J, hidden, hidden, hidden, 2]
    parts = []
    for a, b in zip(dims[:-1], dims[1:]):
        k = 1.0 / np.sqrt(a)
        parts.append(rng.uniform(-k, k, size=(b, a)).reshape(-1))
        parts.append(rng.uniform(-k, k, size=b))
    return np.concatenate(parts).astype(np.float32)


def sample_training_rays(n: int, P: int, V: int, H: int, W: int, hit_mask: Optional[np.ndarray] = None,
                         hit_fraction: float = 0.5, seed: int = 5) -> np.ndarray:
    """Uniform (pose, view, pixel) draws, about `hit_fraction` from hit pixels when a
    boolean hit mask [P][V][H][W] is given.  Returns flat ray ids (int64) into [P][V][H][W]."""
    rng = np.random.default_rng(seed)
    total = P * V * H * W
    if hit_mask is None:
        return rng.integers(0, total, n, dtype=np.int64)
    flat = np.asarray(hit_mask).reshape(-1)
    hits = np.flatnonzero(flat)
    n_hit = int(round(n * hit_fraction)) if len(hits) else 0
    a = hits[rng.integers(0, len(hits), n_hit)] if n_hit else np.zeros(0, dtype=np.int64)
    b = rng.integers(0, total, n - n_hit, dtype=np.int64)
    out = np.concatenate([a, b])
    rng.shuffle(out)
    return out


# (Cout, Cin) of the 14 convolutions of the Light shading network (Cin of the
# first one is the feature width C), then the 1x1 head (4, 32): shapes only,
# for seeding the weights.
def shading_shapes(C: int):
    return [(32, C), (32, 32), (64, 32), (64, 64), (128, 64), (128, 128), (256, 128), (256, 256),
            (128, 384), (128, 128), (64, 192), (64, 64), (32, 96), (32, 32)]


def make_shading_weights(C: int, seed: int = 9) -> np.ndarray:
    """Seeded FP32 weights of the Light shading network in the library's flat
    order: per 3x3 convolution weight [Cout][Cin][3][3] ~ N(0, 2 / (9 Cin))
    (He initialisation) and bias ~ N(0, 0.01^2); then the head weight [4][32]
    ~ N(0, 1/32) and bias [4] = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in shading_shapes(C):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), co * ci * 9))
        parts.append(rng.normal(0.0, 0.01, co))
    parts.append(rng.normal(0.0, math.sqrt(1.0 / 32), 4 * 32))
    parts.append(np.zeros(4))
    return np.concatenate(parts).astype(np.float32)
