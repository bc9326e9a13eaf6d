"""Training-side library calls, through the C ABI:

* art_proposal_io: a network trained K steps, saved, loaded into a fresh
  context and trained K more steps equals, bit for bit, the same network
  trained 2K steps without interruption (the Adam moments and the step count
  travel with the weights; the gradient is deterministic); malformed or
  mismatched files are refused and leave the context as it was.
* art_proposal_calibrate: the margin equals the same quantile computed
  independently in float64 NumPy from the network's outputs and the rays'
  root spans (slab test written out here).
* art_map_loss: dL/dF and dL/dA equal (x - y) * float32(1/R) bit for bit; the
  loss matches the float64 sum of the FP32 differences squared.
* art_proposal_init: the seeded weights equal the oracle's initialisation bit
  for bit and reset the Adam state."""
import os

import numpy as np
import pytest

import scenegen as sg
from gpu_common import log, make_renderer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 3)
    H = W = 48
    K, c2w = sg.make_cameras(s, 2, H, W)
    rend = make_renderer(s, poses, K, c2w, H, W)
    sig = torch.from_numpy(s.sigma).cuda()
    feat = torch.from_numpy(s.feat).cuda()
    lab = rend.proposal_labels(sig, feat, 0.01)
    hit = (lab[..., 0] <= lab[..., 1]).cpu().numpy()
    ids = sg.sample_training_rays(6000, 3, 2, H, W, hit_mask=hit, seed=5)
    od, pose, tgt = rend.proposal_gather(torch.from_numpy(ids).cuda(), lab)
    return dict(s=s, poses=poses, K=K, c2w=c2w, H=H, W=W, rend=rend, od=od, pose=pose, tgt=tgt)


def _fresh(st):
    r = make_renderer(st["s"], st["poses"], st["K"], st["c2w"], st["H"], st["W"])
    r.set_proposal_weights(sg.make_mlp_init(st["s"].J, seed=4))
    return r


def test_proposal_state_resumes_bit_for_bit(setup, tmp_path):
    st = setup
    od, pose, tgt = st["od"], st["pose"], st["tgt"]
    kw = dict(batch=1024, lr=1e-3)
    # uninterrupted: two calls of 12 steps; the interrupted run makes the same
    # two calls with a save and a load in a new context between them
    a = _fresh(st)
    a.proposal_train(od, pose, tgt, steps=12, **kw)
    a.proposal_train(od, pose, tgt, steps=12, **kw)
    wa = a.get_proposal_weights()
    # interrupted after the first call, resumed in a new context
    b = _fresh(st)
    b.proposal_train(od, pose, tgt, steps=12, **kw)
    path = str(tmp_path / "prop.bin")
    b.save_proposal(path)
    assert os.path.getsize(path) == 8 + 8 + 16 + 3 * 4 * b.proposal_param_count()
    c = _fresh(st)
    c.load_proposal(path)
    c.proposal_train(od, pose, tgt, steps=12, **kw)
    wc = c.get_proposal_weights()
    log(f"resume: max |uninterrupted - resumed| = {np.abs(wa - wc).max():.3e}")
    assert np.array_equal(wa, wc)
    # without the moments and step count (weights only) the second call differs
    d = _fresh(st)
    d.set_proposal_weights(b.get_proposal_weights())
    d.proposal_train(od, pose, tgt, steps=12, **kw)
    assert not np.array_equal(wa, d.get_proposal_weights())
    for r in (a, b, c, d):
        r.close()


def test_seeded_init_matches_oracle_and_resets_adam(setup):
    """art_proposal_init(seed): the weights equal the oracle's SplitMix64
    initialisation bit for bit, and a second init with the same seed after
    training restores them with a fresh Adam state (the same training steps
    then give the same weights)."""
    import oracle.mlp as omlp
    import paper_2202_05628_amd as art
    st = setup
    od, pose, tgt = st["od"], st["pose"], st["tgt"]
    J = st["s"].J
    r = make_renderer(st["s"], st["poses"], st["K"], st["c2w"], st["H"], st["W"])
    r.init_proposal(7)
    w0 = r.get_proposal_weights()
    ref = omlp.init_params(J, 7)
    log(f"seeded init: {w0.size} weights, max |library - oracle| = {np.abs(w0 - ref).max():.3e}")
    assert np.array_equal(w0.view(np.uint32), ref.view(np.uint32))
    r.proposal_train(od, pose, tgt, steps=8, batch=1024, lr=1e-3)
    w1 = r.get_proposal_weights()
    assert not np.array_equal(w1, w0)
    r.init_proposal(7)
    assert np.array_equal(r.get_proposal_weights(), w0)
    r.proposal_train(od, pose, tgt, steps=8, batch=1024, lr=1e-3)
    assert np.array_equal(r.get_proposal_weights(), w1)
    r.init_proposal(8)
    assert not np.array_equal(r.get_proposal_weights(), w0)
    r.close()
    # no skeleton: refused
    e = art.Renderer(0)
    with pytest.raises(art.ArtemisError, match="ART_ESTATE"):
        e.init_proposal(1)
    e.close()


def test_proposal_state_refuses_bad_files(setup, tmp_path):
    import paper_2202_05628_amd as art
    st = setup
    r = _fresh(st)
    w0 = r.get_proposal_weights()
    good = str(tmp_path / "good.bin")
    r.save_proposal(good)
    raw = open(good, "rb").read()
    cases = {
        "magic": b"XXXXXXXX" + raw[8:],
        "truncated": raw[:-4],
        "trailing": raw + b"\0",
        "joints": raw[:8] + np.int32(st["s"].J + 1).tobytes() + raw[12:],
        "nan": raw[:32] + np.float32(np.nan).tobytes() + raw[36:],
    }
    for name, data in cases.items():
        p = str(tmp_path / f"{name}.bin")
        open(p, "wb").write(data)
        with pytest.raises(art.ArtemisError) as e:
            r.load_proposal(p)
        assert e.value.status == art._lib.ART_EINVAL, name
        assert np.array_equal(r.get_proposal_weights(), w0), name
    with pytest.raises(art.ArtemisError):
        r.load_proposal(str(tmp_path / "missing.bin"))
    r.close()


def test_calibrated_margin_matches_numpy(setup):
    st = setup
    r = _fresh(st)
    r.proposal_train(st["od"], st["pose"], st["tgt"], steps=30, batch=1024, lr=1e-3)
    od, pose, tgt = st["od"], st["pose"], st["tgt"]
    pred = r.proposal_forward(od, pose).cpu().numpy().astype(np.float64)
    t = tgt.cpu().numpy().astype(np.float64)
    x = od.cpu().numpy().astype(np.float64)
    hit = t[:, 0] <= t[:, 1]
    o, d = x[hit, :3], x[hit, 3:]
    lo = np.full(o.shape[0], -np.inf)
    hi = np.full(o.shape[0], np.inf)
    for a in range(3):
        m = d[:, a] != 0
        t0 = (-1.0 - o[m, a]) / d[m, a]
        t1 = (1.0 - o[m, a]) / d[m, a]
        lo[m] = np.maximum(lo[m], np.minimum(t0, t1))
        hi[m] = np.minimum(hi[m], np.maximum(t0, t1))
    span = hi - np.maximum(lo, 0.0)
    h = 1.0 / (1 << st["s"].depth)
    late = (pred[hit, 0] - t[hit, 0]) * span / h
    for q, floor in [(0.999, 2.0), (0.5, 0.0), (0.9, 0.0), (1.0, 0.0)]:
        ref = max(floor, float(np.quantile(late, q)))
        got = r.calibrate_proposal_margin(od, pose, tgt, quantile=q, floor_h=floor)
        log(f"calibration q={q}: library {got:.5f} numpy {ref:.5f}")
        assert abs(got - ref) <= 1e-4 * max(1.0, abs(ref))
    # a floor above every late start wins
    assert r.calibrate_proposal_margin(od, pose, tgt, quantile=0.5, floor_h=1e6) == 1e6
    r.close()


def test_map_loss_matches_numpy(setup):
    import torch
    st = setup
    r = st["rend"]
    R = r.P * r.V * r.H * r.W
    rng = np.random.default_rng(9)
    C = 8
    F = rng.normal(size=(r.P, r.V, C, r.H, r.W)).astype(np.float32)
    Ft = rng.normal(size=F.shape).astype(np.float32)
    A = rng.uniform(0, 1, size=(r.P, r.V, r.H, r.W)).astype(np.float32)
    At = rng.uniform(0, 1, size=A.shape).astype(np.float32)
    L, dF, dA = r.map_loss(torch.from_numpy(F).cuda(), torch.from_numpy(Ft).cuda(), torch.from_numpy(A).cuda(),
                           torch.from_numpy(At).cuda())
    inv = np.float32(1.0 / R)
    assert np.array_equal(dF.cpu().numpy(), (F - Ft) * inv)
    assert np.array_equal(dA.cpu().numpy(), (A - At) * inv)
    # the differences are taken in FP32 (the maps' precision), squared and summed in FP64
    ref = 0.5 * (((F - Ft).astype(np.float64) ** 2).sum() + ((A - At).astype(np.float64) ** 2).sum()) / R
    assert abs(L - ref) <= 1e-12 * ref
    L2, dF2, dA2 = r.map_loss(torch.from_numpy(F).cuda(), torch.from_numpy(Ft).cuda())
    assert dA2 is None and np.array_equal(dF2.cpu().numpy(), dF.cpu().numpy())
    assert abs(L2 - 0.5 * ((F - Ft).astype(np.float64) ** 2).sum() / R) <= 1e-12 * L2
