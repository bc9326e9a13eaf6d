"""The adjoint's two ways of adding gradients at a launch with many tiles per
workgroup (the full scene, C = 16, 8 poses x 8 cameras at 512x512): by
default the kernel merges the records of one leaf before its atomics; forced
to add them in buffer order it must give the same gradients up to the order
of the float additions.  The merged launch issues fewer additions than it
composites samples; the unmerged one exactly one per sample."""
import numpy as np
import pytest

import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu


def test_merged_gradient_equals_unmerged(monkeypatch):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cfg = sg.CONFIGS["full"]
    s = sg.make_scene(cfg)
    P, V, H, W = 8, 8, cfg.height, cfg.width
    rend = make_renderer(s, sg.make_poses(s.J, P, cfg.pose_seed0), *sg.make_cameras(s, V, H, W), H, W)
    sig, f = flut(s)
    F, A, T = rend.render(sig, f, lambda_th=0.01)
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    dF = torch.randn(F.shape, generator=g, device="cuda") - F
    out = {}
    for mode in ("default", "unmerged"):
        if mode == "unmerged":
            monkeypatch.setenv("ARTEMIS_ADJ_MERGE", "0")
        ds, df = rend.backward(sig, f, F, T, dF, None, lambda_th=0.01, reuse_build=True)
        out[mode] = (ds.cpu().numpy().astype(np.float64), df.cpu().numpy().astype(np.float64), rend.stats())
    (ds0, df0, st0), (ds1, df1, st1) = out["default"], out["unmerged"]
    es = np.abs(ds0 - ds1).max() / np.abs(ds1).max()
    ef = np.abs(df0 - df1).max() / np.abs(df1).max()
    log(f"merge: {st0['samples']} samples, {st0['grad_adds']} merged additions "
        f"({st0['grad_adds'] / st0['samples']:.3f} per sample); dsigma rel_max {es:.2e}, dfeat rel_max {ef:.2e}")
    assert st0["samples"] == st1["samples"] > 10_000_000
    assert st1["grad_adds"] == st1["samples"]
    assert st0["grad_adds"] < 0.9 * st0["samples"]
    assert es <= 1e-5 and ef <= 1e-5
    # the same leaves receive a gradient
    assert np.array_equal(ds0 != 0, ds1 != 0)
