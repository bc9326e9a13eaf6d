"""Pins of the shading-network reference (oracle/shade.py): an independent
NumPy evaluation of the same network (explicit zero padding and shifted sums
for the 3x3 convolutions, reshape-max pooling, repeat upsampling) on tiny
inputs, and the output range."""
import numpy as np

import oracle.shade as osh
import scenegen as sg


HALF = [True]


def _f16(x):
    return x.astype(np.float16).astype(np.float32) if HALF[0] else x.astype(np.float32)


def _conv3(x, W, b):
    """x [C][H][W], W [O][C][3][3]: zero-padded 3x3 cross-correlation as nine
    shifted matrix products, bias, ReLU, FP16 rounding."""
    C, H, Wd = x.shape
    xp = np.zeros((C, H + 2, Wd + 2), np.float32)
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((W.shape[0], H, Wd), np.float64)
    for ky in range(3):
        for kx in range(3):
            y += np.tensordot(W[:, :, ky, kx].astype(np.float64), xp[:, ky:ky + H, kx:kx + Wd].astype(np.float64),
                              axes=(1, 0))
    y += b[:, None, None]
    return _f16(np.maximum(y, 0.0).astype(np.float32))


def _pool(x):
    C, H, W = x.shape
    return x.reshape(C, H // 2, 2, W // 2, 2).max(axis=(2, 4))


def _up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def _numpy_forward(F, w):
    C = F.shape[1]
    layers, (hw, hb) = osh.unpack(w, C)
    Ws = [(_f16(W), b) for W, b in layers]
    out = []
    for img in F:
        x = _f16(img)
        c = lambda i, t: _conv3(t, *Ws[i])
        e0 = c(1, c(0, x))
        e1 = c(3, c(2, _pool(e0)))
        e2 = c(5, c(4, _pool(e1)))
        bt = c(7, c(6, _pool(e2)))
        d2 = c(9, c(8, np.concatenate([e2, _up(bt)])))
        d1 = c(11, c(10, np.concatenate([e1, _up(d2)])))
        d0 = c(13, c(12, np.concatenate([e0, _up(d1)])))
        y = np.tensordot(hw.astype(np.float64), d0.astype(np.float64), axes=(1, 0)) + hb[:, None, None]
        out.append(1.0 / (1.0 + np.exp(-y)))
    return np.stack(out)


def test_reference_matches_independent_numpy_evaluation():
    rng = np.random.default_rng(50)
    C = 5
    F = rng.normal(size=(2, C, 16, 24)).astype(np.float32)
    w = sg.make_shading_weights(C, seed=51)
    # the structure, without FP16 storage: FP32 (torch) against FP64 sums (NumPy)
    HALF[0] = False
    try:
        got32 = osh.forward(F, w, half=False)
        ref32 = _numpy_forward(F, w)
    finally:
        HALF[0] = True
    assert got32.shape == (2, 4, 16, 24)
    assert np.abs(got32 - ref32).max() < 1e-5
    # with FP16 storage: the two sum in different orders, so a stored activation
    # may round to the neighbouring FP16 value and the difference propagates
    got = osh.forward(F, w)
    ref = _numpy_forward(F, w)
    assert np.abs(got - ref).max() < 2e-3
    assert np.median(np.abs(got - ref)) < 2e-4


def test_reference_output_range():
    rng = np.random.default_rng(52)
    F = rng.normal(size=(1, 16, 8, 8)).astype(np.float32)
    y = osh.forward(F, sg.make_shading_weights(16, seed=53))
    assert y.shape == (1, 4, 8, 8) and np.all((y > 0) & (y < 1))
