"""Pins of the oracle's skeleton (FK) and skinning (Eq. 4) against closed forms,
a library rotation routine and exact lattice symmetries (CPU)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen as sg


@pytest.fixture(scope="module")
def tiny():
    return sg.make_scene("tiny")


def _posed_joint(B, rest):
    # posed position of joint j is B_j applied to its rest position
    return np.einsum("jab,jb->ja", B[:, :, :3], rest) + B[:, :, 3]


def test_rodrigues_matches_library(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(200):
        r = rng.normal(size=3) * rng.uniform(0, 3)
        ref = Rotation.from_rotvec(r).as_matrix()
        assert np.allclose(oracle_mod.rodrigues(r), ref, atol=1e-14, rtol=0)
    assert np.array_equal(oracle_mod.rodrigues(np.zeros(3)), np.eye(3))


def test_identity_pose_gives_identity(oracle_mod, tiny):
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, np.zeros((1, tiny.J, 3)), np.zeros((1, 3)),
                      np.zeros((1, 3)))
    eye = np.zeros((3, 4))
    eye[:, :3] = np.eye(3)
    assert np.array_equal(B[0], np.broadcast_to(eye, B[0].shape))


def test_single_joint_rotation(oracle_mod, tiny):
    J = tiny.J
    rest = tiny.rest_joint
    parent = tiny.parent
    j = 2
    r = np.zeros((1, J, 3))
    r[0, j] = [0.1, -0.4, 0.3]
    B = oracle_mod.fk(parent, rest, r, np.zeros((1, 3)), np.zeros((1, 3)))[0]
    Rj = Rotation.from_rotvec(r[0, j]).as_matrix()
    # descendants of j (including j)
    desc = set([j])
    for k in range(J):
        if parent[k] in desc:
            desc.add(k)
    pj = _posed_joint(B, rest)
    for k in range(J):
        if k in desc:
            assert np.allclose(B[k, :, :3], Rj, atol=1e-14)
            assert np.allclose(pj[k], rest[j] + Rj @ (rest[k] - rest[j]), atol=1e-14)
        else:
            assert np.allclose(B[k], np.hstack([np.eye(3), np.zeros((3, 1))]), atol=0)
    assert np.allclose(pj[j], rest[j], atol=1e-15)


def test_bone_lengths_preserved(oracle_mod, tiny):
    r, R, T = sg.make_poses(tiny.J, 4)
    R = np.array([[0.3, -0.2, 0.5]] * 4)
    T = np.array([[0.01, 0.02, -0.03]] * 4)
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, r, R, T)
    for p in range(4):
        pj = _posed_joint(B[p], tiny.rest_joint)
        for k in range(1, tiny.J):
            a = np.linalg.norm(pj[k] - pj[tiny.parent[k]])
            b = np.linalg.norm(tiny.rest_joint[k] - tiny.rest_joint[tiny.parent[k]])
            assert abs(a - b) < 1e-14
        for k in range(tiny.J):
            Rk = B[p, k, :, :3]
            assert np.allclose(Rk.T @ Rk, np.eye(3), atol=1e-14)
            assert abs(np.linalg.det(Rk) - 1.0) < 1e-14


def test_global_rotation_about_root(oracle_mod, tiny):
    Rv = np.array([0.2, 0.5, -0.1])
    Tv = np.array([0.05, 0.0, 0.1])
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, np.zeros((1, tiny.J, 3)), Rv[None], Tv[None])[0]
    Rm = Rotation.from_rotvec(Rv).as_matrix()
    J0 = tiny.rest_joint[0]
    for k in range(tiny.J):
        assert np.allclose(B[k, :, :3], Rm, atol=1e-14)
        assert np.allclose(B[k, :, 3], J0 - Rm @ J0 + Tv, atol=1e-14)


def test_identity_pose_cells_shift(oracle_mod, tiny):
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, np.zeros((1, tiny.J, 3)), np.zeros((1, 3)),
                      np.zeros((1, 3)))
    pt = oracle_mod.lbs(tiny.ijk, tiny.depth, tiny.bone, tiny.weight, B[0])
    cells, valid = oracle_mod.posed_cells(pt, tiny.depth)
    assert valid.all()
    assert np.array_equal(cells, tiny.ijk.T.astype(np.int64) + (1 << (tiny.depth - 1)))


def test_integer_translation_shifts_keys(oracle_mod, tiny):
    h = 1.0 / (1 << tiny.depth)
    k = np.array([3, -2, 5])
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, np.zeros((1, tiny.J, 3)), np.zeros((1, 3)),
                      (k * h)[None])
    pt = oracle_mod.lbs(tiny.ijk, tiny.depth, tiny.bone, tiny.weight, B[0])
    cells, valid = oracle_mod.posed_cells(pt, tiny.depth)
    assert valid.all()
    assert np.array_equal(cells, tiny.ijk.T.astype(np.int64) + (1 << (tiny.depth - 1)) + k)


def test_quarter_turn_permutes_cells(oracle_mod, tiny):
    # +90 degrees about z through the root joint (the origin, a lattice corner):
    # (x, y, z) -> (-y, x, z) maps cell (cx, cy, cz) to (G - 1 - cy, cx, cz)
    G = 1 << (tiny.depth + 1)
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, np.zeros((1, tiny.J, 3)),
                      np.array([[0.0, 0.0, math.pi / 2]]), np.zeros((1, 3)))
    pt = oracle_mod.lbs(tiny.ijk, tiny.depth, tiny.bone, tiny.weight, B[0])
    cells, valid = oracle_mod.posed_cells(pt, tiny.depth)
    c0 = tiny.ijk.T.astype(np.int64) + (1 << (tiny.depth - 1))
    expect = np.stack([G - 1 - c0[:, 1], c0[:, 0], c0[:, 2]], axis=1)
    assert valid.all()
    assert np.array_equal(cells, expect)


def test_single_bone_is_rigid(oracle_mod, tiny):
    r, R, T = sg.make_poses(tiny.J, 1)
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, r, R, T)[0]
    n = 300
    ijk = tiny.ijk[:, :n]
    bone = np.zeros((4, n), dtype=np.uint8)
    bone[0] = 5
    w = np.zeros((4, n), dtype=np.float32)
    w[0] = 1.0
    pt = oracle_mod.lbs(ijk, tiny.depth, bone, w, B)
    pc = oracle_mod.canonical_centres(ijk, tiny.depth)
    d0 = np.linalg.norm(pc[:, None] - pc[None], axis=-1)
    d1 = np.linalg.norm(pt[:, None] - pt[None], axis=-1)
    assert np.allclose(d0, d1, atol=1e-14)


def test_matrix_blend_equals_point_blend(oracle_mod, tiny):
    r, R, T = sg.make_poses(tiny.J, 1)
    B = oracle_mod.fk(tiny.parent, tiny.rest_joint, r, R, T)[0]
    pt = oracle_mod.lbs(tiny.ijk, tiny.depth, tiny.bone, tiny.weight, B)
    pc = oracle_mod.canonical_centres(tiny.ijk, tiny.depth)
    ref = np.zeros_like(pc)
    for k in range(4):
        Bk = B[tiny.bone[k].astype(int)]
        ref += tiny.weight[k].astype(np.float64)[:, None] * (
            np.einsum("nab,nb->na", Bk[:, :, :3], pc) + Bk[:, :, 3])
    assert np.allclose(pt, ref, atol=1e-14)
