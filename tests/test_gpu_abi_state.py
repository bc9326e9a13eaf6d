"""Boundary behaviour of the C ABI that keeps a context consistent:

* a render whose tile lists overflowed re-runs the overflowed (pose, view
  group) items; an adjoint that asks to reuse that render's posed octrees must
  then rebuild them and give the gradients of one that rebuilds;
* the autograd backward refuses to run after the poses (or cameras) changed
  since its forward render;
* negative or non-finite FLUT densities are refused (ART_EINVAL), and the
  context renders correctly afterwards;
* a working-memory limit below one pose's needs gives ART_ENOMEM, and the
  context renders correctly afterwards; a limit that holds fewer poses than a
  call asks for makes the call render in several batches, with the same maps.
"""
import os

import numpy as np
import pytest

import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

REL = 1e-5   # summation-order rounding of the adjoint's atomic accumulation


def _same(a, b):
    return float((a - b).abs().max()) <= REL * float(b.abs().max()) + 1e-30


@pytest.fixture(scope="module")
def tiny():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 3)
    K, c2w = sg.make_cameras(s, 2, 80, 72)
    return s, poses, K, c2w


def test_overflow_rerun_then_reused_backward(tiny, monkeypatch):
    import torch
    s, poses, K, c2w = tiny
    monkeypatch.setenv("ARTEMIS_PAIR_CAP", "64")   # every tile list overflows on the first attempt
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    sig, f = flut(s)
    F, A, T = rend.render(sig, f, 0.01)
    monkeypatch.delenv("ARTEMIS_PAIR_CAP")
    ref = make_renderer(s, poses, K, c2w, 80, 72)
    F0, A0, T0 = ref.render(sig, f, 0.01)
    assert torch.equal(F, F0) and torch.equal(A, A0) and torch.equal(T, T0)
    dF = torch.randn_like(F)
    d1 = rend.backward(sig, f, F, T, dF, lambda_th=0.01, reuse_build=True)
    n1 = rend.stats()["launches"]
    d0 = rend.backward(sig, f, F, T, dF, lambda_th=0.01, reuse_build=False)
    n0 = rend.stats()["launches"]
    log(f"overflow re-run: reused backward {n1} launches, rebuilt {n0}")
    assert n1 == n0                    # the partly re-run build is not reused
    assert _same(d1[0], d0[0]) and _same(d1[1], d0[1])
    assert float(d0[0].abs().max()) > 0


def test_autograd_backward_after_new_poses_raises(tiny):
    import torch
    import paper_2202_05628_amd as art
    s, poses, K, c2w = tiny
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    sig, f = flut(s)
    sig.requires_grad_(True)
    F, A = art.render(rend, sig, f, lambda_th=0.01)
    rend.set_poses(*sg.make_poses(s.J, 3, seed0=2000))
    with pytest.raises(art.ArtemisError) as e:
        (F ** 2).sum().backward()
    assert e.value.status == -4   # ART_ESTATE
    # forward, new poses, forward again: the first graph's backward still refuses
    sig.grad = None
    F1, _ = art.render(rend, sig, f, lambda_th=0.01)
    rend.set_poses(*poses)
    F2, _ = art.render(rend, sig, f, lambda_th=0.01)
    with pytest.raises(art.ArtemisError):
        (F1 ** 2).sum().backward()
    (F2 ** 2).sum().backward()        # the current graph works
    assert float(sig.grad.abs().max()) > 0


@pytest.mark.parametrize("bad", [-1.0, float("nan"), float("inf")])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_invalid_density_rejected(tiny, bad, storage):
    import torch
    import paper_2202_05628_amd as art
    s, poses, K, c2w = tiny
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    sig, f = flut(s, storage)
    F0, A0, T0 = rend.render(sig, f, 0.01)
    sb = sig.clone()
    sb[123] = bad
    with pytest.raises(art.ArtemisError) as e:
        rend.render(sb, f, 0.01)
    assert e.value.status == -1   # ART_EINVAL
    with pytest.raises(art.ArtemisError):
        rend.backward(sb, f, F0, T0, torch.ones_like(F0), lambda_th=0.01)
    F1, A1, T1 = rend.render(sig, f, 0.01)
    assert torch.equal(F1, F0) and torch.equal(A1, A0) and torch.equal(T1, T0)


def test_memory_limit(tiny):
    import torch
    import paper_2202_05628_amd as art
    s, poses, K, c2w = tiny
    sig, f = flut(s)
    ref = make_renderer(s, poses, K, c2w, 80, 72)
    F0, A0, T0 = ref.render(sig, f, 0.01)
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    rend.set_memory_limit(1 << 20)   # below one pose's posed octree and tile lists
    with pytest.raises(art.ArtemisError) as e:
        rend.render(sig, f, 0.01)
    assert e.value.status == -2   # ART_ENOMEM
    assert rend.memory()["working_bytes"] <= (1 << 20)
    rend.set_memory_limit(0)
    F1, A1, T1 = rend.render(sig, f, 0.01)
    assert torch.equal(F1, F0) and torch.equal(A1, A0) and torch.equal(T1, T0)
    whole = rend.memory()["working_bytes"]
    log(f"memory limit: one call of 3 poses holds {whole} working bytes")
    # a fresh context bounded to about half of that renders the poses in batches
    small = make_renderer(s, poses, K, c2w, 80, 72)
    small.set_memory_limit(whole * 6 // 10)
    F2, A2, T2 = small.render(sig, f, 0.01)
    assert torch.equal(F2, F0) and torch.equal(A2, A0) and torch.equal(T2, T0)
    assert small.memory()["working_bytes"] <= whole * 6 // 10
