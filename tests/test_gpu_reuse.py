"""Reuse of the posed octrees and tile lists that a render call leaves in the
library's scratch slots (ART_REUSE_BUILD), for the adjoint and the VRT term.

They depend on the octree, skin, skeleton, poses, cameras and the geometry
precision only, so an adjoint or VRT call that reuses them must give the
gradients of one that rebuilds them.  Both add their gradients with float
atomics, whose order varies from run to run, so "the same" is to within the
rounding of that order (REL of the largest entry); the number of kernel
launches shows whether the build was skipped.  Any change of those inputs
since the render (here new poses, or the other geometry precision) must make
the call rebuild."""
import numpy as np
import pytest

import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu

REL = 1e-5   # summation-order rounding of the atomic accumulation


def _same(a, b):
    import torch
    return float((a - b).abs().max()) <= REL * float(b.abs().max()) + 1e-30


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    posesA = sg.make_poses(s.J, 2)
    posesB = sg.make_poses(s.J, 2, seed0=2000)
    K, c2w = sg.make_cameras(s, 2, 64, 72)
    rend = make_renderer(s, posesA, K, c2w, 64, 72)
    return s, rend, posesA, posesB


def _backward(rend, sig, f, F, T, dF, reuse, fp32=False):
    import torch
    ds = torch.zeros_like(sig)
    df = torch.zeros_like(f)
    rend.backward(sig, f, F, T, dF, lambda_th=0.01, fp32_geom=fp32, d_sigma=ds, d_feat=df, reuse_build=reuse)
    return ds, df, rend.stats()["launches"]


@pytest.mark.parametrize("fp32", [False, True])
def test_backward_reuse_is_bitwise_and_skips_the_build(setup, fp32):
    import torch
    s, rend, posesA, _ = setup
    rend.set_poses(*posesA)
    sig, f = flut(s)
    F, A, T = rend.render(sig, f, 0.01, fp32_geom=fp32)
    dF = torch.randn_like(F)
    ds1, df1, n1 = _backward(rend, sig, f, F, T, dF, reuse=True, fp32=fp32)
    ds0, df0, n0 = _backward(rend, sig, f, F, T, dF, reuse=False, fp32=fp32)
    log(f"backward fp32={fp32}: launches with reuse {n1}, rebuilt {n0}")
    assert _same(ds1, ds0) and _same(df1, df0)
    assert n1 < n0
    # the rebuild just done leaves valid octrees again: a second reuse matches too
    ds2, df2, n2 = _backward(rend, sig, f, F, T, dF, reuse=True, fp32=fp32)
    assert _same(ds2, ds0) and _same(df2, df0) and n2 == n1


def test_reuse_after_new_poses_rebuilds(setup):
    import torch
    s, rend, posesA, posesB = setup
    sig, f = flut(s)
    rend.set_poses(*posesB)
    FB, _, TB = rend.render(sig, f, 0.01)
    dF = torch.randn_like(FB)
    ds0, df0, n0 = _backward(rend, sig, f, FB, TB, dF, reuse=False)
    rend.set_poses(*posesA)
    rend.render(sig, f, 0.01)            # leaves the octrees of poses A
    rend.set_poses(*posesB)              # ... which no longer apply
    ds1, df1, n1 = _backward(rend, sig, f, FB, TB, dF, reuse=True)
    log(f"reuse after set_poses: launches {n1} (rebuilt: {n0})")
    assert n1 == n0
    assert _same(ds1, ds0) and _same(df1, df0)


def test_reuse_with_other_geometry_precision_rebuilds(setup):
    import torch
    s, rend, posesA, _ = setup
    rend.set_poses(*posesA)
    sig, f = flut(s)
    F, _, T = rend.render(sig, f, 0.01, fp32_geom=False)
    dF = torch.randn_like(F)
    ds0, df0, n0 = _backward(rend, sig, f, F, T, dF, reuse=False, fp32=True)
    rend.render(sig, f, 0.01, fp32_geom=False)   # FP64-geometry octrees
    ds1, df1, n1 = _backward(rend, sig, f, F, T, dF, reuse=True, fp32=True)
    assert n1 == n0
    assert _same(ds1, ds0) and _same(df1, df0)


def test_vrt_reuse_is_bitwise(setup):
    import torch
    s, rend, posesA, posesB = setup
    sig, f = flut(s)
    for poses in (posesA, posesB):
        rend.set_poses(*poses)
        rend.render(sig, f, 0.01)
        l1, d1 = rend.vrt(f, 0.05, reuse_build=True)
        l0, d0 = rend.vrt(f, 0.05)
        l2, d2 = rend.vrt(f, 0.05, reuse_build=True)   # after a VRT rebuild: no tile lists, rebuilt again
        log(f"vrt reuse: loss {l1:.6e} vs {l0:.6e}")
        assert abs(l1 - l0) <= REL * abs(l0) and abs(l2 - l0) <= REL * abs(l0)
        assert _same(d1, d0) and _same(d2, d0)
    # new poses after the render: the VRT must rebuild
    rend.set_poses(*posesA)
    rend.render(sig, f, 0.01)
    rend.set_poses(*posesB)
    l3, d3 = rend.vrt(f, 0.05, reuse_build=True)
    l4, d4 = rend.vrt(f, 0.05)
    assert abs(l3 - l4) <= REL * abs(l4) and _same(d3, d4)
