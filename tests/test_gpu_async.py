"""ART_ASYNC: render calls that only enqueue their work, with the overflow and
density checks reported afterwards by art_render_status.

* An asynchronous render gives the synchronous render's maps bit for bit
  once the stream is synchronised, and the same run statistics.
* With tile lists too small for the call (ARTEMIS_PAIR_CAP), the
  asynchronous call leaves the overflowed items unrendered and the status
  reports them; the next call has grown the lists and renders them right.
* A negative or non-finite density makes an asynchronous call render nothing
  without an error; the status counts the bad densities.
* A call that needs several pose batches stays synchronous; ART_ASYNC with
  ART_TIMING is refused.
"""
import numpy as np
import pytest

import scenegen as sg
from gpu_common import flut, log, make_renderer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    s = sg.make_scene("tiny")
    poses = sg.make_poses(s.J, 3)
    K, c2w = sg.make_cameras(s, 2, 80, 72)
    return s, poses, K, c2w


def _ref(tiny):
    s, poses, K, c2w = tiny
    sig, f = flut(s)
    ref = make_renderer(s, poses, K, c2w, 80, 72)
    out = ref.render(sig, f, 0.01)
    return out, ref.stats()


def test_async_render_equals_sync(tiny):
    import torch
    s, poses, K, c2w = tiny
    (F0, A0, T0), st0 = _ref(tiny)
    sig, f = flut(s)
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    for _ in range(2):   # a fresh context, then one with grown buffers
        F, A, T = rend.render(sig, f, 0.01, sync=False)
        torch.cuda.synchronize()
        assert torch.equal(F, F0) and torch.equal(A, A0) and torch.equal(T, T0)
        assert rend.render_status() == {"overflowed_items": 0, "bad_densities": 0}
        st = rend.stats()
        for k in ("rays", "samples", "hit_rays", "rounds", "steps", "tile_rays"):
            assert st[k] == st0[k], k
    # after a synchronous call the status has nothing to report
    rend.render(sig, f, 0.01)
    assert rend.render_status() == {"overflowed_items": 0, "bad_densities": 0}


def test_async_overflow_is_reported_and_fixed_by_the_next_call(tiny, monkeypatch):
    import torch
    s, poses, K, c2w = tiny
    (F0, A0, T0), _ = _ref(tiny)
    sig, f = flut(s)
    monkeypatch.setenv("ARTEMIS_PAIR_CAP", "64")   # every tile list overflows
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    F, A, T = rend.render(sig, f, 0.01, sync=False)
    monkeypatch.delenv("ARTEMIS_PAIR_CAP")
    status = rend.render_status()
    log(f"async with 64-entry tile lists: {status}")
    assert status["overflowed_items"] > 0 and status["bad_densities"] == 0
    F, A, T = rend.render(sig, f, 0.01, sync=False)
    assert rend.render_status() == {"overflowed_items": 0, "bad_densities": 0}
    assert torch.equal(F, F0) and torch.equal(A, A0) and torch.equal(T, T0)


def test_async_bad_density_is_reported(tiny):
    import torch
    import paper_2202_05628_amd as art
    s, poses, K, c2w = tiny
    sig, f = flut(s)
    bad = sig.clone()
    bad[7] = float("nan")
    bad[11] = -1.0
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    rend.render(bad, f, 0.01, sync=False)
    assert rend.render_status() == {"overflowed_items": 0, "bad_densities": 2}
    with pytest.raises(art.ArtemisError) as e:
        rend.render(bad, f, 0.01)
    assert e.value.status == art._lib.ART_EINVAL


def test_async_several_batches_and_flags(tiny):
    import torch
    import paper_2202_05628_amd as art
    s, poses, K, c2w = tiny
    (F0, A0, T0), _ = _ref(tiny)
    sig, f = flut(s)
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    rend.render(sig, f, 0.01)
    whole = rend.memory()["working_bytes"]
    small = make_renderer(s, poses, K, c2w, 80, 72)
    small.set_memory_limit(whole * 6 // 10)   # the 3 poses take several batches: the call is synchronous
    F, A, T = small.render(sig, f, 0.01, sync=False)
    assert torch.equal(F, F0) and torch.equal(A, A0) and torch.equal(T, T0)
    assert small.render_status() == {"overflowed_items": 0, "bad_densities": 0}
    with pytest.raises(art.ArtemisError) as e:
        rend.render(sig, f, 0.01, timing=True, sync=False)
    assert e.value.status == art._lib.ART_EINVAL


def test_async_render_leaves_a_reusable_build(tiny):
    """After an asynchronous render whose status reports nothing, a reusing
    adjoint (ART_REUSE_BUILD) skips the build and gives the rebuilt adjoint's
    gradients; without the status call nothing is reused."""
    import torch
    s, poses, K, c2w = tiny
    sig, f = flut(s)
    rend = make_renderer(s, poses, K, c2w, 80, 72)
    F, A, T = rend.render(sig, f, 0.01, sync=False)
    assert rend.render_status() == {"overflowed_items": 0, "bad_densities": 0}
    dF = torch.randn_like(F)

    def grads(reuse):
        ds, df = rend.backward(sig, f, F, T, dF, lambda_th=0.01, reuse_build=reuse)
        return ds, df, rend.stats()["launches"]

    ds1, df1, n1 = grads(True)
    ds0, df0, n0 = grads(False)
    log(f"async render then adjoint: {n1} launches reusing the build, {n0} rebuilding")
    assert n1 < n0
    rel = lambda a, b: float((a - b).abs().max()) / float(b.abs().max())
    assert rel(ds1, ds0) <= 1e-5 and rel(df1, df0) <= 1e-5
    # the status never read: the build is not taken as complete
    rend.render(sig, f, 0.01, sync=False)
    _, _, n2 = grads(True)
    assert n2 == n0
