"""The Light shading network on the matrix cores against the PyTorch reference
(oracle/shade.py: FP32 convolutions on FP16-rounded weights and activations).

Both sides store every activation in FP16 and accumulate in FP32, but in
different orders, so a stored activation can land on the neighbouring FP16
value; the difference propagates through the remaining layers.  The bar is
5e-3 absolute on the sigmoid outputs (in [0, 1]) with a median below 5e-4;
the reference's own FP32-vs-FP64 structure check is in test_oracle_shade.py."""
import numpy as np
import pytest

import oracle.shade as osh
import scenegen as sg
from gpu_common import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rend():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2202_05628_amd as art
    return art.Renderer(0)


# widths 512 and 1024 take the widest tiles (64 pixels x 64 channels per wave,
# waves over pixels and channels) at every level, as the 512^2 maps do; the
# 512 x 512 map is the benchmark's own shape (every level's full row count)
@pytest.mark.parametrize("C,N,H,W", [(16, 2, 32, 48), (16, 1, 24, 136), (8, 3, 16, 16), (16, 1, 16, 264), (32, 1, 16, 32),
                                     (4, 2, 8, 72), (16, 1, 16, 512), (12, 1, 8, 1024), (16, 1, 512, 512)])
def test_shading_matches_reference(rend, C, N, H, W):
    import torch
    rng = np.random.default_rng(60 + C + W)
    F = rng.normal(size=(N, C, H, W)).astype(np.float32)
    F[:, :, : H // 4, :] = 0.0           # a background band, as rendered maps have
    w = sg.make_shading_weights(C, seed=61)
    rend.set_shading_weights(C, w)
    out = rend.shade(torch.from_numpy(F).cuda()).cpu().numpy()
    ref = osh.forward(F, w)
    d = np.abs(out - ref)
    log(f"shading C={C} N={N} {H}x{W}: max |diff| {d.max():.2e}, median {np.median(d):.2e}")
    assert out.shape == (N, 4, H, W)
    assert d.max() < 5e-3 and np.median(d) < 5e-4


def test_shading_argument_errors(rend):
    import paper_2202_05628_amd as art
    import torch
    rend.set_shading_weights(16, sg.make_shading_weights(16))
    with pytest.raises(art.ArtemisError):
        rend.shade(torch.zeros((1, 16, 12, 16), device="cuda"))      # H not a multiple of 8
    with pytest.raises(art.ArtemisError):
        rend.shade(torch.zeros((1, 8, 16, 16), device="cuda"))       # weights are for C = 16
    with pytest.raises(art.ArtemisError):
        rend.set_shading_weights(16, np.zeros(10, dtype=np.float32))


def test_fused_head_equals_separate_head(rend, monkeypatch):
    """The head fused into the last convolution (default) against the separate
    head kernel (ARTEMIS_SHADE_HEAD=0): the same FP16 activations enter both,
    so the outputs differ only by the order of the 32-term FP32 sums."""
    import torch
    rng = np.random.default_rng(77)
    F = torch.from_numpy(rng.normal(size=(2, 16, 40, 264)).astype(np.float32)).cuda()
    rend.set_shading_weights(16, sg.make_shading_weights(16, seed=61))
    fused = rend.shade(F)
    monkeypatch.setenv("ARTEMIS_SHADE_HEAD", "0")
    separate = rend.shade(F)
    monkeypatch.delenv("ARTEMIS_SHADE_HEAD")
    d = (fused - separate).abs().max().item()
    log(f"fused head vs separate head kernel: max |diff| {d:.2e}")
    assert d <= 1e-6
