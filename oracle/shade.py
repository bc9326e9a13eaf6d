"""Reference of the "Light" neural shading network (plain PyTorch on the CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Section 3.1 ("Neural
Shading") converts the feature map F into an image with a U-Net; the runtime
analysis (Tab. 5) names a "Light" variant without the opacity branch, whose
appearance branch predicts the opacity as one more output channel, run in half
precision.  The paper gives neither widths nor depths; the readings (stated
again where the library documents its entry points):

* four encoder levels of 32, 64, 128 and 256 channels, two 3x3 convolutions
  (padding 1, bias, ReLU) each, 2x2 max pooling between levels;
* three decoder levels of 128, 64 and 32 channels: the first convolution of a
  level reads the concatenation [encoder output of that level, nearest 2x
  upsampling of the level below], the second refines it;
* a 1x1 head to 4 channels (R, G, B, opacity) and a sigmoid;
* half precision as stored values: the input, the weights and every
  activation are rounded to FP16; products accumulate in FP32; the head is
  FP32.

The weights come flat in the library's order (``scenegen.make_shading_weights``).
"""
from __future__ import annotations

import numpy as np

SHAPES_TAIL = [(32, 32), (64, 32), (64, 64), (128, 64), (128, 128), (256, 128), (256, 256),
               (128, 384), (128, 128), (64, 192), (64, 64), (32, 96), (32, 32)]


def unpack(w: np.ndarray, C: int):
    """Per-layer (weight [Cout][Cin][3][3], bias) of the 14 convolutions and the
    head (weight [4][32], bias [4]) from the flat parameter vector."""
    shapes = [(32, C)] + SHAPES_TAIL
    out, p = [], 0
    for co, ci in shapes:
        W = w[p:p + co * ci * 9].reshape(co, ci, 3, 3)
        p += co * ci * 9
        b = w[p:p + co]
        p += co
        out.append((W, b))
    hw = w[p:p + 128].reshape(4, 32)
    p += 128
    hb = w[p:p + 4]
    assert p + 4 == w.size
    return out, (hw, hb)


def forward(F: np.ndarray, w: np.ndarray, half: bool = True) -> np.ndarray:
    """F [N][C][H][W] (H, W multiples of 8) -> [N][4][H][W].  half=False keeps
    every stored value in FP32 (the network's arithmetic without the FP16
    storage, for checking the structure)."""
    import torch
    import torch.nn.functional as Fn
    _h = (lambda x: x.half().float()) if half else (lambda x: x)
    C = F.shape[1]
    layers, (hw, hb) = unpack(np.asarray(w, dtype=np.float32), C)
    Wt = [(_h(torch.from_numpy(np.ascontiguousarray(W))), torch.from_numpy(np.ascontiguousarray(b)))
          for W, b in layers]

    def conv(i, x):
        W, b = Wt[i]
        return _h(torch.relu(Fn.conv2d(x, W, b, padding=1)))

    x = _h(torch.from_numpy(np.ascontiguousarray(F, dtype=np.float32)))
    e0 = conv(1, conv(0, x))
    e1 = conv(3, conv(2, Fn.max_pool2d(e0, 2)))
    e2 = conv(5, conv(4, Fn.max_pool2d(e1, 2)))
    bt = conv(7, conv(6, Fn.max_pool2d(e2, 2)))
    d2 = conv(9, conv(8, torch.cat([e2, Fn.interpolate(bt, scale_factor=2, mode="nearest")], dim=1)))
    d1 = conv(11, conv(10, torch.cat([e1, Fn.interpolate(d2, scale_factor=2, mode="nearest")], dim=1)))
    d0 = conv(13, conv(12, torch.cat([e0, Fn.interpolate(d1, scale_factor=2, mode="nearest")], dim=1)))
    y = torch.einsum("oc,nchw->nohw", torch.from_numpy(hw), d0) + torch.from_numpy(hb)[None, :, None, None]
    return torch.sigmoid(y).numpy()
