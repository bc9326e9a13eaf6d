"""Pins of the oracle's ray-interval proposal: its labels (entry of the first
and exit of the last composited sample) against an all-voxel slab test on tiny
grids and a hand-derived worked example, and its FP64 network against central
finite differences, an independent automatic-differentiation implementation
(torch, float64), torch's SmoothL1 and Adam, and a library rotation routine."""
import json
import math
import os

import numpy as np
import pytest

import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _slab(o, d, lo, hi):
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if o[a] < lo[a] or o[a] > hi[a]:
                return 1.0, 0.0
            continue
        u = (lo[a] - o[a]) / d[a]
        v = (hi[a] - o[a]) / d[a]
        t0 = max(t0, min(u, v))
        t1 = min(t1, max(u, v))
    return t0, t1


def _brute_interval(o, d, depth, cells):
    """(t_a, t_b, first entry, last exit) over every occupied cell whose slab
    overlap with the clipped ray has positive length (lambda_th = 0: every such
    cell is composited)."""
    h = 1.0 / (1 << depth)
    ta, tb = _slab(o, d, -np.ones(3), np.ones(3))
    ta = max(ta, 0.0)
    if not tb > ta:
        return None
    first, last = np.inf, -np.inf
    for c in cells:
        lo = -1.0 + c * h
        t0, t1 = _slab(o, d, lo, lo + h)
        t0, t1 = max(t0, ta), min(t1, tb)
        if t1 > t0:
            first = min(first, t0)
            last = max(last, t1)
    return ta, tb, first, last


@pytest.mark.parametrize("depth,frac", [(1, 0.3), (2, 0.1), (3, 0.02)])
def test_labels_equal_brute_force(oracle_mod, depth, frac):
    rng = np.random.default_rng(40 + depth)
    G = 1 << (depth + 1)
    occ = rng.random((G, G, G)) < frac
    cz, cy, cx = np.nonzero(occ.transpose(2, 1, 0))
    cells = np.stack([cx, cy, cz], axis=1)
    lin = (cells[:, 2] * G + cells[:, 1]) * G + cells[:, 0]
    order = np.argsort(lin)
    lin, cells = lin[order], cells[order]
    n = len(lin)
    o = rng.uniform(-2.5, 2.5, (400, 3))
    d = rng.uniform(-0.9, 0.9, (400, 3)) - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = oracle_mod.render(o, d, depth, lin, np.arange(n), np.ones(n), np.zeros((n, 1)), 0.0)
    lab = oracle_mod.interval_labels(out["seg"])
    h = 1.0 / (1 << depth)
    checked = hits = 0
    for r in range(len(o)):
        if out["min_gap"][r] < 1e-9 * h:
            continue
        ref = _brute_interval(o[r], d[r], depth, cells)
        if ref is None:
            assert np.isnan(out["seg"][r, 0]) and tuple(lab[r]) == (1.0, 0.0)
            continue
        ta, tb, first, last = ref
        assert abs(out["seg"][r, 0] - ta) < 1e-12 and abs(out["seg"][r, 1] - tb) < 1e-12
        if not np.isfinite(first):
            assert out["n_comp"][r] == 0 and tuple(lab[r]) == (1.0, 0.0)
        else:
            hits += 1
            assert abs(out["seg"][r, 2] - first) < 1e-12 and abs(out["seg"][r, 3] - last) < 1e-12
            assert abs(lab[r, 0] - (first - ta) / (tb - ta)) < 1e-12
            assert abs(lab[r, 1] - (last - ta) / (tb - ta)) < 1e-12
            assert 0.0 <= lab[r, 0] < lab[r, 1] <= 1.0
        checked += 1
    assert checked > 350 and hits > 50


def test_labels_golden_column(oracle_mod):
    with open(os.path.join(GOLDEN, "two_voxel_column.json")) as fh:
        g = json.load(fh)
    depth = g["depth"]
    G = 1 << (depth + 1)
    c = np.array(g["cells"])
    lin = (c[:, 2] * G + c[:, 1]) * G + c[:, 0]
    sig = np.array(g["sigma_over_ln2"]) * math.log(2.0)
    f = np.array(g["feat"])
    for case in g["cases"]:
        out = oracle_mod.render(np.array([g["ray_origin"]]), np.array([g["ray_dir"]]), depth, lin,
                                np.array(g["leaf_ids"]), sig, f, case["lambda_th"])
        lab = oracle_mod.interval_labels(out["seg"])[0]
        assert np.allclose(lab, case["interval"], rtol=0, atol=1e-15)


def test_labels_stop_at_early_termination(oracle_mod):
    # a column of 6 dense voxels: with lambda_th the last composited sample is
    # the one at which T first drops below the threshold
    depth = 2
    G = 8
    cells = np.array([[x, 3, 3] for x in range(1, 7)])
    lin = (cells[:, 2] * G + cells[:, 1]) * G + cells[:, 0]
    h = 0.25
    sig = np.full(6, math.log(4.0) / h)   # each voxel: alpha = 3/4, T *= 1/4
    o = np.array([[-3.0, -1 + 3.5 * h, -1 + 3.5 * h]])
    d = np.array([[1.0, 0.0, 0.0]])
    for lam, n in ((0.0, 6), (0.1, 2), (0.3, 1), (0.01, 4)):
        out = oracle_mod.render(o, d, depth, lin, np.arange(6), sig, np.zeros((6, 1)), lam)
        assert out["n_comp"][0] == n
        ta, tb = 2.0, 4.0
        lab = oracle_mod.interval_labels(out["seg"])[0]
        # cell x = k spans t in [t_a + k h, t_a + (k + 1) h]
        assert abs(lab[0] - h / (tb - ta)) < 1e-15
        assert abs(lab[1] - (1 + n) * h / (tb - ta)) < 1e-15


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

def _problem(J=2, n=32, seed=0):
    import oracle.mlp as mlp
    rng = np.random.default_rng(seed)
    theta = sg.make_mlp_init(J, seed=seed + 1).astype(np.float64)
    # push the pre-activations away from 0 so finite differences do not cross a ReLU kink
    X = np.concatenate([rng.normal(size=(n, 6)), rng.uniform(-1, 1, (n, 6 * J))], axis=1)
    t = rng.uniform(0, 1, (n, 2))
    return mlp, theta, X, t


def test_mlp_shapes():
    import oracle.mlp as mlp
    assert mlp.param_count(40) == 24258
    assert mlp.param_count(12) == 64 * 78 + 64 + 2 * (64 * 64 + 64) + 2 * 64 + 2
    assert sg.make_mlp_init(40).size == 24258


def test_splitmix64_published_outputs():
    """The generator of the seeded initialisation against the first five
    outputs of SplitMix64 for seed 1234567 as listed in the Rosetta Code task
    "Pseudo-random numbers/Splitmix64"."""
    import oracle.mlp as mlp
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    assert [mlp.splitmix64(1234567, k) for k in range(1, 6)] == want


def test_seeded_init_ranges_and_moments():
    """Every layer's values lie in (-1/sqrt(fan-in), 1/sqrt(fan-in)) with the
    mean and spread of that uniform distribution; seeds give different draws."""
    import oracle.mlp as mlp
    J = 40
    a, b = mlp.init_params(J, 7), mlp.init_params(J, 8)
    assert a.dtype == np.float32 and a.size == mlp.param_count(J)
    assert np.array_equal(a, mlp.init_params(J, 7)) and not np.array_equal(a, b)
    p = mlp.unpack(a.astype(np.float64), J)
    for name in ("W1", "W2", "W3"):
        k = 1.0 / math.sqrt(p[name].shape[1])
        w = p[name].reshape(-1)
        assert np.abs(w).max() < k
        assert abs(w.mean()) < 0.02 * k and abs(w.std() / (k / math.sqrt(3.0)) - 1.0) < 0.03


def test_mlp_gradient_finite_differences():
    mlp, theta, X, t = _problem()
    L, g = mlp.grad(theta, X, t, 2)
    _, act = mlp.forward(theta, X, 2)
    rng = np.random.default_rng(3)
    idx = rng.choice(theta.size, 300, replace=False)
    eps = 1e-6
    fd = np.empty(len(idx))
    for k, i in enumerate(idx):
        tp = theta.copy()
        tp[i] += eps
        tm = theta.copy()
        tm[i] -= eps
        fd[k] = (mlp.loss(mlp.forward(tp, X, 2)[0], t) - mlp.loss(mlp.forward(tm, X, 2)[0], t)) / (2 * eps)
    err = np.abs(fd - g[idx]).max() / np.abs(g[idx]).max()
    assert err < 1e-6, err


def test_mlp_gradient_matches_torch_autograd():
    import torch
    mlp, theta, X, t = _problem(J=3, n=50, seed=5)
    L, g = mlp.grad(theta, X, t, 3)
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(theta, 3).items()}
    x = torch.tensor(X)
    h = torch.relu(torch.nn.functional.linear(x, p["W1"], p["b1"]))
    h = torch.relu(torch.nn.functional.linear(h, p["W2"], p["b2"]))
    h = torch.relu(torch.nn.functional.linear(h, p["W3"], p["b3"]))
    y = torch.sigmoid(torch.nn.functional.linear(h, p["W4"], p["b4"]))
    lt = torch.nn.functional.smooth_l1_loss(y, torch.tensor(t), beta=1.0)
    lt.backward()
    gt = np.concatenate([p[k].grad.numpy().reshape(-1) for k, _ in mlp.param_shapes(3)])
    assert abs(lt.item() - L) < 1e-14
    assert np.abs(gt - g).max() <= 1e-12 * np.abs(gt).max()
    assert np.allclose(y.detach().numpy(), mlp.forward(theta, X, 3)[0], rtol=0, atol=1e-14)


def test_smooth_l1_matches_torch():
    import torch
    import oracle.mlp as mlp
    e = np.linspace(-3, 3, 61)
    ref = torch.nn.functional.smooth_l1_loss(torch.tensor(e), torch.zeros(61, dtype=torch.float64),
                                             reduction="none", beta=1.0).numpy()
    assert np.allclose(mlp.smooth_l1(e), ref, rtol=0, atol=1e-15)


def test_adam_matches_torch():
    import torch
    import oracle.mlp as mlp
    rng = np.random.default_rng(8)
    theta = rng.normal(size=40)
    grads = [rng.normal(size=40) * 10 ** rng.uniform(-3, 1) for _ in range(6)]
    w = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(40)
    v = np.zeros(40)
    for k, g in enumerate(grads):
        w.grad = torch.tensor(g)
        opt.step()
        theta, m, v = mlp.adam_step(theta, m, v, g, k + 1)
    assert np.abs(w.detach().numpy() - theta).max() < 1e-14


def test_pose_code_is_two_rotation_columns():
    from scipy.spatial.transform import Rotation
    import oracle.mlp as mlp
    r, _, _ = sg.make_poses(5, 3)
    code = mlp.pose_code(r)
    for p in range(3):
        for j in range(5):
            M = Rotation.from_rotvec(r[p, j]).as_matrix()
            assert np.allclose(code[p, 6 * j:6 * j + 6], np.concatenate([M[:, 0], M[:, 1]]), atol=1e-14)
    assert np.array_equal(mlp.pose_code(np.zeros((1, 4, 3))), np.tile([1.0, 0, 0, 0, 1, 0], (1, 4)))


def test_bf16_forms_close_to_fp64():
    mlp, theta, X, t = _problem(J=4, n=64, seed=9)
    y64 = mlp.forward(theta, X, 4)[0]
    y16 = mlp.forward(theta, X, 4, precision="bf16")[0]
    y48 = mlp.forward(theta, X, 4, precision="bf16x3")[0]
    assert np.abs(y64 - y16).max() < 2e-2
    assert np.abs(y64 - y48).max() < 1e-4
    _, g64 = mlp.grad(theta, X, t, 4)
    _, g16 = mlp.grad(theta, X, t, 4, precision="bf16")
    _, g48 = mlp.grad(theta, X, t, 4, precision="bf16x3")
    assert np.abs(g64 - g16).max() / np.abs(g64).max() < 5e-2
    assert np.abs(g64 - g48).max() / np.abs(g64).max() < 1e-3


def test_bf16x3_product_is_near_exact():
    import oracle.mlp as mlp
    rng = np.random.default_rng(12)
    a = rng.normal(size=(40, 64))
    b = rng.normal(size=(64, 30))
    ref = a @ b
    err = np.abs(mlp._mm(a, b, "bf16x3") - ref).max() / np.abs(ref).max()
    err1 = np.abs(mlp._mm(a, b, "bf16") - ref).max() / np.abs(ref).max()
    assert err < 2e-5 < err1


def test_pinball_minimiser_is_the_quantile():
    """Over a constant prediction the pinball loss at level tau is smallest at
    the tau-quantile of the targets: brute force over every order statistic
    (the minimum of a piecewise-linear convex function lies at one of its
    breakpoints)."""
    import oracle.mlp as mlp
    rng = np.random.default_rng(14)
    t = rng.uniform(0.0, 1.0, 501)
    ts = np.sort(t)
    for tau in (0.01, 0.1, 0.5, 0.9, 0.99):
        losses = [mlp.pinball(t - c, tau).mean() for c in ts]
        best = ts[int(np.argmin(losses))]
        # the tau-quantile: the smallest order statistic with at least tau of the mass at or below it
        k = int(np.ceil(tau * len(t))) - 1
        assert best == ts[k], (tau, best, ts[k])


def test_pinball_half_is_half_the_absolute_error():
    import oracle.mlp as mlp
    rng = np.random.default_rng(15)
    y = rng.uniform(0, 1, (50, 2))
    t = np.sort(rng.uniform(0, 1, (50, 2)), axis=1)     # labels with a sample: u_near <= u_far
    assert np.allclose(mlp.loss(y, t, "pinball", (0.5, 0.5)), 0.5 * np.abs(y - t).mean(), rtol=0, atol=1e-15)
    # one-sided weights: a prediction above the target costs 1 - tau per unit
    assert np.isclose(mlp.loss(np.array([[0.7, 0.2]]), np.array([[0.5, 0.5]]), "pinball", (0.1, 0.9)),
                      0.5 * ((1 - 0.1) * 0.2 + 0.9 * 0.3))
    # rays with the empty label (1, 0) keep SmoothL1
    ye = np.array([[0.3, 0.6]])
    te = np.array([[1.0, 0.0]])
    assert np.isclose(mlp.loss(ye, te, "pinball", (0.01, 0.99)), mlp.loss(ye, te))


def test_mlp_pinball_gradient_finite_differences():
    mlp, theta, X, t = _problem(J=3, n=40, seed=16)
    t[::3] = (1.0, 0.0)   # every third ray with the empty label
    assert (t[:, 0] <= t[:, 1]).sum() > 5
    tau = (0.02, 0.97)
    L, g = mlp.grad(theta, X, t, 3, kind="pinball", tau=tau)
    rng = np.random.default_rng(17)
    eps = 1e-6
    for i in rng.choice(theta.size, 40, replace=False):
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        lp = mlp.loss(mlp.forward(tp, X, 3)[0], t, "pinball", tau)
        lm = mlp.loss(mlp.forward(tm, X, 3)[0], t, "pinball", tau)
        assert abs((lp - lm) / (2 * eps) - g[i]) <= 1e-7 * max(1.0, np.abs(g).max()), i
