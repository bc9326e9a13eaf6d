"""Pins of the oracle's adjoint: central finite differences of its own FP64
forward and the single-voxel closed form (CPU)."""
import math

import numpy as np
import pytest

import scenegen as sg


@pytest.fixture(scope="module")
def setup(oracle_mod):
    s = sg.make_scene("tiny")
    r, R, T = sg.make_poses(s.J, 1)
    B = oracle_mod.fk(s.parent, s.rest_joint, r, R, T)[0]
    ok, ol, _, _, _ = oracle_mod.pose_occupancy(s.ijk, s.depth, s.bone, s.weight, B)
    K, c2w = sg.make_cameras(s, 1, 40, 40)
    o, d = oracle_mod.camera_rays(K, c2w, 40, 40)
    o, d = o.reshape(-1, 3), d.reshape(-1, 3)
    rng = np.random.default_rng(3)
    target = rng.normal(size=(len(o), s.C))
    a_w = rng.normal(size=len(o))
    return s, ok, ol, o, d, target, a_w


def _loss(oracle_mod, setup, sigma, feat, lam):
    s, ok, ol, o, d, target, a_w = setup
    out = oracle_mod.render(o, d, s.depth, ok, ol, sigma, feat, lam)
    return 0.5 * np.sum((out["F"] - target) ** 2) + np.sum(a_w * out["A"]), out


def test_gradient_matches_central_differences(oracle_mod, setup):
    s, ok, ol, o, d, target, a_w = setup
    sigma = s.sigma.astype(np.float64)
    feat = s.feat.astype(np.float64)
    L, out = _loss(oracle_mod, setup, sigma, feat, 0.0)
    gF = out["F"] - target
    dsig, dfeat = oracle_mod.backward(o, d, s.depth, ok, ol, sigma, feat, 0.0, gF, a_w)
    visible = np.nonzero(dsig != 0)[0]
    assert len(visible) > 200
    rng = np.random.default_rng(5)
    pick = rng.choice(visible, 24, replace=False)
    eps = 1e-3
    for leaf in pick:
        sp = sigma.copy(); sp[leaf] += eps
        sm = sigma.copy(); sm[leaf] -= eps
        fd = (_loss(oracle_mod, setup, sp, feat, 0.0)[0] - _loss(oracle_mod, setup, sm, feat, 0.0)[0]) / (2 * eps)
        assert abs(fd - dsig[leaf]) <= 1e-6 * max(1.0, abs(dsig[leaf]))
        c = int(rng.integers(0, s.C))
        fp = feat.copy(); fp[leaf, c] += eps
        fm = feat.copy(); fm[leaf, c] -= eps
        fd = (_loss(oracle_mod, setup, sigma, fp, 0.0)[0] - _loss(oracle_mod, setup, sigma, fm, 0.0)[0]) / (2 * eps)
        assert abs(fd - dfeat[leaf, c]) <= 1e-7 * max(1.0, abs(dfeat[leaf, c]))
    # leaves that no ray reaches, and collision losers, get exactly zero
    assert np.all(dsig[np.setdiff1d(np.arange(s.n), ol)] == 0)


def test_gradient_with_early_stop_holds_samples_fixed(oracle_mod, setup):
    s, ok, ol, o, d, target, a_w = setup
    sigma = s.sigma.astype(np.float64)
    feat = s.feat.astype(np.float64)
    lam = 0.01
    L, out = _loss(oracle_mod, setup, sigma, feat, lam)
    dsig, dfeat = oracle_mod.backward(o, d, s.depth, ok, ol, sigma, feat, lam,
                                      out["F"] - target, a_w)
    rng = np.random.default_rng(8)
    visible = np.nonzero(dsig != 0)[0]
    eps = 1e-4
    checked = 0
    for leaf in rng.choice(visible, 40, replace=False):
        sp = sigma.copy(); sp[leaf] += eps
        sm = sigma.copy(); sm[leaf] -= eps
        Lp, op = _loss(oracle_mod, setup, sp, feat, lam)
        Lm, om = _loss(oracle_mod, setup, sm, feat, lam)
        if not (np.array_equal(op["n_comp"], out["n_comp"]) and np.array_equal(om["n_comp"], out["n_comp"])):
            continue   # the perturbation moved a stop sample: not differentiable there
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - dsig[leaf]) <= 1e-5 * max(1.0, abs(dsig[leaf]))
        checked += 1
    assert checked >= 20


def test_single_voxel_opacity_derivative(oracle_mod):
    depth = 2
    G = 1 << (depth + 1)
    h = 1.0 / (1 << depth)
    cell = np.array([2, 5, 3])
    lin = np.array([(cell[2] * G + cell[1]) * G + cell[0]])
    o = np.array([[-2.0, -1.0 + 5.4 * h, -1.0 + 3.7 * h]])
    d = np.array([[1.0, 0.02, -0.01]])
    d /= np.linalg.norm(d)
    sig = np.array([6.0])
    f = np.array([[0.0]])
    out = oracle_mod.render(o, d, depth, lin, np.array([0]), sig, f, 0.0, max_hits=2)
    ell = out["hit_delta"][0, 0]
    dsig, _ = oracle_mod.backward(o, d, depth, lin, np.array([0]), sig, f, 0.0,
                                  np.zeros((1, 1)), np.ones(1))
    assert abs(dsig[0] - ell * math.exp(-sig[0] * ell)) < 1e-15
