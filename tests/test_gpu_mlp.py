"""The proposal network's own GPU kernels against the FP64 oracle network.

Inputs are computed by the oracle (rays of the cameras in FP64, cast to FP32;
pose codes from the axis-angles) and handed to the GPU; the GPU's outputs,
loss, gradients and Adam updates are compared with
  (a) the oracle in plain FP64 (the 1e-2 bar of the BF16 matrix-core forms),
  (b) the oracle's emulation of the GPU's operand rounding: single BF16
      operands for the network outputs (inference form), split BF16 operands
      (head + tail, three products) for the loss gradient (training form);
      this bar is tight.
A ragged ray count (not a multiple of the 256-ray gradient chunk) exercises the
padding; the gradient is deterministic (fixed-order partial sums)."""
import numpy as np
import pytest

import oracle
import oracle.mlp as omlp
import scenegen as sg
from gpu_common import log, make_renderer

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-2      # BF16 matrix-core forms vs the FP64 network
TOL_FORM = 2e-3      # vs the oracle's emulation of the same operand rounding


@pytest.fixture(scope="module")
def net():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 5)
    H = W = 64
    K, c2w = sg.make_cameras(s, 3, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    theta = sg.make_mlp_init(s.J)
    rend.set_proposal_weights(theta)
    o, d = oracle.camera_rays(K, c2w, H, W)
    code = omlp.pose_code(poses[0])
    rng = np.random.default_rng(31)
    n = 1000
    ids = rng.integers(0, 5 * 3 * H * W, n)
    p = ids // (3 * H * W)
    v = (ids // (H * W)) % 3
    pix = ids % (H * W)
    od = np.concatenate([o[v, pix // W, pix % W], d[v, pix // W, pix % W]], axis=1).astype(np.float32)
    tgt = rng.uniform(0, 1, (n, 2)).astype(np.float32)
    X = omlp.inputs(od[:, :3].astype(np.float64), od[:, 3:].astype(np.float64), code[p])
    dev = dict(od=torch.from_numpy(od).cuda(), pose=torch.from_numpy(p.astype(np.int32)).cuda(),
               tgt=torch.from_numpy(tgt).cuda())
    return dict(s=s, rend=rend, theta=theta.astype(np.float64), X=X, tgt=tgt.astype(np.float64), dev=dev, ids=ids,
                K=K, c2w=c2w, poses=poses, H=H, W=W)


def _rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_forward_matches_oracle(net):
    rend, dev = net["rend"], net["dev"]
    log("proposal forward: 1000 rays, J=12")
    y = rend.proposal_forward(dev["od"], dev["pose"]).cpu().numpy().astype(np.float64)
    J = net["s"].J
    y64 = omlp.forward(net["theta"], net["X"], J)[0]
    y16 = omlp.forward(net["theta"], net["X"], J, precision="bf16")[0]
    log(f"  vs fp64 {_rel_max(y, y64):.2e}  vs bf16 form {_rel_max(y, y16):.2e}")
    assert _rel_max(y, y16) <= TOL_FORM
    assert _rel_max(y, y64) <= TOL_FP64


def test_gradient_matches_oracle(net):
    rend, dev = net["rend"], net["dev"]
    J = net["s"].J
    L, g = rend.proposal_grad(dev["od"], dev["pose"], dev["tgt"])
    g = g.cpu().numpy().astype(np.float64)
    L64, g64 = omlp.grad(net["theta"], net["X"], net["tgt"], J)
    L48, g48 = omlp.grad(net["theta"], net["X"], net["tgt"], J, precision="bf16x3")
    parts = omlp.unpack(g, J)
    p64 = omlp.unpack(g64, J)
    p48 = omlp.unpack(g48, J)
    errs = {k: (_rel_max(parts[k], p64[k]), _rel_max(parts[k], p48[k])) for k in p64}
    for k, (e64, e48) in errs.items():
        log(f"  d{k}: vs fp64 {e64:.2e}  vs bf16x3 form {e48:.2e}")
    for k, (e64, e48) in errs.items():
        assert e48 <= TOL_FORM, k
        assert e64 <= TOL_FP64, k
    assert abs(L - L64) <= 1e-4 * L64 and abs(L - L48) <= 1e-4 * L48


def test_gradient_is_deterministic(net):
    rend, dev = net["rend"], net["dev"]
    _, g1 = rend.proposal_grad(dev["od"], dev["pose"], dev["tgt"])
    _, g2 = rend.proposal_grad(dev["od"], dev["pose"], dev["tgt"])
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())


def test_adam_step_matches_oracle(net):
    rend, dev = net["rend"], net["dev"]
    J = net["s"].J
    theta0 = net["theta"]
    rend.set_proposal_weights(theta0.astype(np.float32))
    lr = 1e-3
    losses = rend.proposal_train(dev["od"], dev["pose"], dev["tgt"], batch=1000, steps=1, lr=lr)
    theta1 = rend.get_proposal_weights().astype(np.float64)
    _, g48 = omlp.grad(theta0, net["X"], net["tgt"], J, precision="bf16x3")
    ref, _, _ = omlp.adam_step(theta0, np.zeros_like(theta0), np.zeros_like(theta0), g48, 1, lr=lr)
    dg, dr = theta1 - theta0, ref - theta0
    firm = np.abs(g48) >= 1e-3 * np.abs(g48).max()   # gradients well above the rounding noise
    log(f"  adam: {firm.sum()} firm params, max |d - d_ref| {np.abs(dg - dr)[firm].max():.2e}")
    assert np.abs(dg - dr)[firm].max() <= 2e-2 * lr
    assert np.abs(dg).max() <= 1.001 * lr
    assert abs(losses[0] - omlp.loss(omlp.forward(theta0, net["X"], J)[0], net["tgt"])) < 1e-2 * losses[0]
    rend.set_proposal_weights(theta0.astype(np.float32))


def test_gather_matches_oracle_rays(net):
    import torch
    rend = net["rend"]
    s = net["s"]
    H, W = net["H"], net["W"]
    sig = torch.from_numpy(s.sigma).cuda()
    f = torch.from_numpy(s.feat).cuda()
    lab = rend.proposal_labels(sig, f, 0.01)
    ids = torch.from_numpy(net["ids"]).cuda()
    od, pose, tgt = rend.proposal_gather(ids, lab)
    o, d = oracle.camera_rays(net["K"], net["c2w"], H, W)
    ids_np = net["ids"]
    v = (ids_np // (H * W)) % 3
    pix = ids_np % (H * W)
    ref = np.concatenate([o[v, pix // W, pix % W], d[v, pix // W, pix % W]], axis=1)
    assert np.abs(od.cpu().numpy() - ref).max() < 1e-5
    assert np.array_equal(pose.cpu().numpy(), ids_np // (3 * H * W))
    assert np.array_equal(tgt.cpu().numpy(), lab.reshape(-1, 2)[ids].cpu().numpy())


def test_argument_errors(net):
    import paper_2202_05628_amd as art
    import torch
    rend, dev = net["rend"], net["dev"]
    bad = dev["pose"].clone()
    bad[7] = 99
    with pytest.raises(art.ArtemisError):
        rend.proposal_forward(dev["od"], bad)
    with pytest.raises(art.ArtemisError):
        rend.set_proposal_weights(np.zeros(5, dtype=np.float32))
    with pytest.raises(art.ArtemisError):
        rend.proposal_gather(torch.tensor([-1], dtype=torch.int64, device="cuda"),
                             torch.zeros((5, 3, 64, 64, 2), device="cuda"))


def test_training_lowers_the_loss_and_guides_the_traversal(net):
    """Train on labels of the plain renderer (seeded rays, about half with a
    composited sample) with the one-sided loss (pinball at levels 0.03 / 0.97
    on rays with a sample, SmoothL1 on empty labels), calibrate the start
    margin on held-out rays (99 % of the late starts covered), then render
    with the network's intervals (front skipping only).  Gain criterion: the
    guided render takes fewer partition steps than the plain render with the
    error against it within 1e-3 (rel_mean).  The trained network meets it;
    the untrained network, calibrated by the same rule, does not (its margin
    covers the whole front: no step is saved).  The wave rounds are not
    asserted: the lanes that fall back (F1) cost the tile a second pass over
    its brick list, which on this scene outweighs the saved steps."""
    import torch
    rend, s = net["rend"], net["s"]
    sig = torch.from_numpy(s.sigma).cuda()
    f = torch.from_numpy(s.feat).cuda()
    lab = rend.proposal_labels(sig, f, 0.01)
    hit = (lab[..., 0] <= lab[..., 1]).cpu().numpy()
    ids = sg.sample_training_rays(60000, rend.P, rend.V, rend.H, rend.W, hit_mask=hit, seed=5)
    od, pose, tgt = rend.proposal_gather(torch.from_numpy(ids).cuda(), lab)
    F0, _, _ = rend.render(sig, f, 0.01)
    steps0 = rend.stats()["steps"]
    theta0 = sg.make_mlp_init(s.J)
    val = slice(54000, None)

    def guided(q=0.99):
        m = rend.calibrate_proposal_margin(od[val], pose[val], tgt[val], quantile=q)
        Fg, _, _ = rend.render_proposal(sig, f, None, 0.01, margin_h=m, near_only=True)
        st = rend.stats()
        return m, float((Fg - F0).abs().sum() / F0.abs().sum()), st["steps"], st

    rend.set_proposal_loss("pinball", (0.03, 0.97))
    rend.set_proposal_weights(theta0)
    mu, err_u, steps_u, _ = guided()
    L0, _ = rend.proposal_grad(od[val], pose[val], tgt[val])
    log_ = rend.proposal_train(od[:54000], pose[:54000], tgt[:54000], batch=4096, steps=6000, lr=3e-3)
    L1, _ = rend.proposal_grad(od[val], pose[val], tgt[val])
    log(f"  train loss {log_[0]:.4f} -> {log_[-1]:.4f}; validation {L0:.4f} -> {L1:.4f}")
    assert L1 < 0.3 * L0
    mt, err, steps_t, st = guided()
    log(f"  trained: margin {mt:.2f} h, rel_mean {err:.2e}, steps {steps_t} vs plain {steps0} "
        f"(fallbacks {st['fallbacks']} of {st['proposal_rays']}); untrained: margin {mu:.2f} h, "
        f"rel_mean {err_u:.2e}, steps {steps_u}")
    assert err <= 1e-3 and steps_t < steps0          # the trained network saves work within the bar
    assert not (err_u <= 1e-3 and steps_u < steps0)  # the control does not
    assert steps_u == steps0
    # start estimates of the held-out hit rays: trained vs untrained network
    hitv = (tgt[val, 0] <= tgt[val, 1]).cpu().numpy()
    yt = rend.proposal_forward(od[val], pose[val]).cpu().numpy()
    trained = rend.get_proposal_weights()
    rend.set_proposal_weights(theta0)
    yu = rend.proposal_forward(od[val], pose[val]).cpu().numpy()
    rend.set_proposal_weights(trained)
    rend.set_proposal_loss("smooth_l1")
    tv = tgt[val].cpu().numpy()
    # the pinball level 0.03 asks for late starts on about 3 % of the rays
    late_t = float((yt[hitv, 0] > tv[hitv, 0]).mean())
    late_u = float((yu[hitv, 0] > tv[hitv, 0]).mean())
    over_t = float(np.maximum(yt[hitv, 0] - tv[hitv, 0], 0.0).mean())
    over_u = float(np.maximum(yu[hitv, 0] - tv[hitv, 0], 0.0).mean())
    log(f"  held-out hit rays starting late: trained {late_t:.4f} (mean late part {over_t:.5f}), "
        f"untrained {late_u:.4f} ({over_u:.5f})")
    assert late_t <= 0.1
    assert over_t < 0.5 * over_u


def test_pinball_gradient_matches_oracle(net):
    """The one-sided loss (pinball on rays with a sample, SmoothL1 on empty
    labels) and its gradient on the GPU against the oracle network, in FP64
    and in the oracle's emulation of the split-BF16 training products."""
    import torch
    rend, dev = net["rend"], net["dev"]
    J = net["s"].J
    tau = (0.05, 0.9)
    tgt = net["tgt"].copy()
    tgt[::4] = (1.0, 0.0)   # every fourth ray with the empty label
    rend.set_proposal_weights(net["theta"].astype(np.float32))   # the fixture's weights (earlier tests train)
    rend.set_proposal_loss("pinball", tau)
    try:
        L, g = rend.proposal_grad(dev["od"], dev["pose"], torch.from_numpy(tgt.astype(np.float32)).cuda())
    finally:
        rend.set_proposal_loss("smooth_l1")
    g = g.cpu().numpy().astype(np.float64)
    L64, g64 = omlp.grad(net["theta"], net["X"], tgt, J, kind="pinball", tau=tau)
    L48, g48 = omlp.grad(net["theta"], net["X"], tgt, J, precision="bf16x3", kind="pinball", tau=tau)
    log(f"pinball loss {L:.6f} vs oracle {L64:.6f}; gradient vs fp64 {_rel_max(g, g64):.2e}, "
        f"vs split form {_rel_max(g, g48):.2e}")
    assert abs(L - L64) <= 1e-4 * abs(L64)
    assert _rel_max(g, g48) <= TOL_FORM
    assert _rel_max(g, g64) <= TOL_FP64


@pytest.mark.parametrize("H,W", [(64, 64), (40, 52)])
def test_render_inference_matches_network_forward(net, H, W):
    """The guided render evaluates the network itself for the rays of every
    non-empty tile; handing it the outputs of art_proposal_forward for the
    same rays (inputs from art_proposal_gather) must give the same maps bit for
    bit.  This pins the pixel of each inference lane (tile, 16-ray group,
    shuffle of the ray inputs), also for ragged tiles (W = 52)."""
    import torch
    from gpu_common import flut
    s = net["s"]
    poses = net["poses"]
    K, c2w = sg.make_cameras(s, 2, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    theta = sg.make_mlp_init(s.J)
    theta[-2:] = [-0.85, 0.85]   # output biases: intervals around [0.3, 0.7] of each span, varying per ray
    rend.set_proposal_weights(theta)
    sig, f = flut(s)
    P, V = len(poses[0]), 2
    lab = rend.proposal_labels(sig, f, 0.01)
    ids = torch.arange(P * V * H * W, dtype=torch.int64, device="cuda")
    od, pose, _ = rend.proposal_gather(ids, lab)
    iv = rend.proposal_forward(od, pose).reshape(P, V, H, W, 2)
    kw = dict(margin_h=2.0, f2_tau=-1.0)
    Fa, Aa, Ta = rend.render_proposal(sig, f, None, 0.01, **kw)
    st_a = rend.stats()
    Fb, Ab, Tb = rend.render_proposal(sig, f, iv, 0.01, **kw)
    st_b = rend.stats()
    log(f"inference in the render vs network forward {H}x{W}: proposal rays {st_a['proposal_rays']}, "
        f"fallbacks {st_a['fallbacks']} / {st_b['fallbacks']}")
    assert st_a["proposal_rays"] > 0
    assert torch.equal(Fa, Fb) and torch.equal(Aa, Ab) and torch.equal(Ta, Tb)
    assert st_a["proposal_rays"] == st_b["proposal_rays"] and st_a["fallbacks"] == st_b["fallbacks"]
    assert st_a["rounds"] == st_b["rounds"]
    # control: the intervals of the neighbouring pixel change the maps, so the
    # comparison above does see which pixel an interval belongs to
    Fc, _, _ = rend.render_proposal(sig, f, torch.roll(iv, 1, dims=3).contiguous(), 0.01, **kw)
    assert not torch.equal(Fa, Fc)
