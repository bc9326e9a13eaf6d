"""Pins of the oracle's posed octree: occupied set, min-id collision winners and
the 8^3-brick level, against vectorised set constructions (CPU)."""
import numpy as np
import pytest

import scenegen as sg


def _morton(c):
    key = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(10):
        for a in range(3):
            key |= ((c[:, a] >> b) & 1) << (3 * b + a)
    return key


@pytest.fixture(scope="module")
def posed(oracle_mod):
    s = sg.make_scene("tiny")
    r, R, T = sg.make_poses(s.J, 1)
    B = oracle_mod.fk(s.parent, s.rest_joint, r, R, T)[0]
    pt = oracle_mod.lbs(s.ijk, s.depth, s.bone, s.weight, B)
    cells, valid = oracle_mod.posed_cells(pt, s.depth)
    return s, cells, valid


def test_morton_matches_bitwise_definition(oracle_mod):
    rng = np.random.default_rng(1)
    c = rng.integers(0, 1024, size=(500, 3))
    key = oracle_mod.morton30(c)
    for i in range(500):
        k = int(key[i])
        for a in range(3):
            back = sum(((k >> (3 * b + a)) & 1) << b for b in range(10))
            assert back == c[i, a]


def test_occupied_set_and_winners(oracle_mod, posed):
    s, cells, valid = posed
    keys = oracle_mod.posed_keys(cells, valid)
    oc = oracle_mod.posed_octree(keys)
    # np.unique returns the first index of each value: the minimum leaf id
    u, first = np.unique(keys[valid], return_index=True)
    leaf_ids = np.nonzero(valid)[0]
    assert np.array_equal(oc["keys"], u.astype(np.uint32))
    assert np.array_equal(oc["winner"], leaf_ids[first])
    # collisions happen in this pose, so the winner rule is exercised
    assert len(u) < valid.sum()
    # every winner's own key is the cell it wins
    assert np.array_equal(keys[oc["winner"]], oc["keys"])


def test_brick_level(oracle_mod, posed):
    s, cells, valid = posed
    keys = oracle_mod.posed_keys(cells, valid)
    oc = oracle_mod.posed_octree(keys)
    occ = oc["keys"].astype(np.int64)
    bricks = np.unique(occ >> 9)
    assert np.array_equal(oc["brick_keys"].astype(np.int64), bricks)
    # mask bit set iff the leaf cell is occupied; row base is the first leaf of the brick
    occ_set = set(occ.tolist())
    for b, bk in enumerate(bricks.tolist()):
        for local in range(512):
            bit = (int(oc["brick_mask"][b, local >> 5]) >> (local & 31)) & 1
            assert bit == (((bk << 9) | local) in occ_set)
        r = int(oc["brick_row"][b])
        assert occ[r] >> 9 == bk and (r == 0 or occ[r - 1] >> 9 != bk)


def test_dropped_leaves_counted(oracle_mod):
    cells = np.array([[0, 0, 0], [5, 5, 5], [-1, 2, 2], [128, 0, 0]])
    valid = np.array([True, True, False, False])
    keys = oracle_mod.posed_keys(cells, valid)
    oc = oracle_mod.posed_octree(keys)
    assert oc["dropped"] == 2
    assert list(oc["winner"]) == [0, 1]


def test_linear_and_morton_occupancy_agree(oracle_mod, posed):
    s, cells, valid = posed
    G = 1 << (s.depth + 1)
    lin, win = oracle_mod.occupancy_from_cells(cells, valid, s.depth)
    c = np.stack([lin % G, (lin // G) % G, lin // (G * G)], axis=1)
    m = _morton(c)
    order = np.argsort(m)
    oc = oracle_mod.posed_octree(oracle_mod.posed_keys(cells, valid))
    assert np.array_equal(m[order].astype(np.uint32), oc["keys"])
    assert np.array_equal(win[order], oc["winner"])


def test_identity_pose_equals_canonical_occupancy(oracle_mod):
    s = sg.make_scene("tiny")
    B = oracle_mod.fk(s.parent, s.rest_joint, np.zeros((1, s.J, 3)), np.zeros((1, 3)),
                      np.zeros((1, 3)))[0]
    k1, l1, _, _, _ = oracle_mod.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B)
    k2, l2 = oracle_mod.canonical_occupancy(s.ijk, s.depth)
    assert np.array_equal(k1, k2) and np.array_equal(l1, l2)
    assert len(k1) == s.n
