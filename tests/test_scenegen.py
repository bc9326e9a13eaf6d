"""Seeded synthetic inputs: sizes, validity and reproducibility (CPU)."""
import numpy as np
import pytest

import scenegen as sg


@pytest.fixture(scope="module")
def tiny():
    return sg.make_scene("tiny")


def _morton(ijk, bits):
    key = np.zeros(ijk.shape[1], dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            key |= ((ijk[a].astype(np.int64) >> b) & 1) << (3 * b + a)
    return key


def test_leaf_count_and_range(tiny):
    assert abs(tiny.n - 20_000) <= 0.02 * 20_000
    G = 1 << tiny.depth
    assert tiny.ijk.dtype == np.uint16 and tiny.ijk.shape == (3, tiny.n)
    assert int(tiny.ijk.max()) < G
    key = _morton(tiny.ijk, tiny.depth)
    assert np.all(np.diff(key) > 0), "leaves unique and in canonical Morton order"


def test_skin_weights(tiny):
    assert tiny.bone.shape == (4, tiny.n) and tiny.weight.shape == (4, tiny.n)
    assert int(tiny.bone.max()) < tiny.J
    s = tiny.weight.astype(np.float64).sum(axis=0)
    assert np.all(np.abs(s - 1.0) < 1e-6)
    assert np.all(tiny.weight > 0)
    # the four bone ids of a leaf are distinct
    b = np.sort(tiny.bone.astype(int), axis=0)
    assert np.all(np.diff(b, axis=0) > 0)


def test_skeleton_tree(tiny):
    p = tiny.parent
    assert p[0] == -1 and np.all(p[1:] >= 0) and np.all(p[1:] < np.arange(1, len(p)))
    # root joint at the origin, a lattice corner
    assert np.all(tiny.rest_joint[0] == 0.0)


def test_appearance(tiny):
    assert tiny.sigma.min() >= 5.0 and tiny.sigma.max() <= 50.0
    assert tiny.feat.shape == (tiny.n, 8)
    assert abs(float(tiny.feat.mean())) < 0.05 and abs(float(tiny.feat.std()) - 1.0) < 0.05


def test_reproducible(tiny):
    again = sg.make_scene("tiny")
    assert np.array_equal(tiny.ijk, again.ijk)
    assert np.array_equal(tiny.weight, again.weight)
    assert np.array_equal(tiny.feat, again.feat)
    r1 = sg.make_poses(tiny.J, 3)
    r2 = sg.make_poses(tiny.J, 3)
    assert all(np.array_equal(a, b) for a, b in zip(r1, r2))


def test_poses_within_30_degrees(tiny):
    r, R, T = sg.make_poses(tiny.J, 5)
    ang = np.linalg.norm(r, axis=-1)
    assert ang.max() <= np.radians(30.0) + 1e-12
    assert np.all(R == 0) and np.all(T == 0)


def test_cameras_look_at_centre(tiny):
    K, c2w = sg.make_cameras(tiny, 4, 64, 48)
    for v in range(4):
        Rm = c2w[v, :, :3]
        assert np.allclose(Rm.T @ Rm, np.eye(3), atol=1e-12)
        assert np.isclose(np.linalg.det(Rm), 1.0)
        fwd = tiny.centre - c2w[v, :, 3]
        assert np.allclose(Rm[:, 2], fwd / np.linalg.norm(fwd))
        assert K[v, 0, 2] == 24.0 and K[v, 1, 2] == 32.0
