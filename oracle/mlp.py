"""FP64 reference of the learned ray-interval proposal network.

TEST INFRASTRUCTURE ONLY (see the package docstring): the plain definition the
GPU network kernels are checked against.  The proposal is an addition to the
paper's renderer, not part of it; what it predicts is defined by the
renderer's composited samples (Section 3.1, Eq. 5 and Eq. 6): for a ray with
span [t_a, t_b] inside the posed root, the entry t of its first and the exit t
of its last composited sample, mapped to [0, 1] (``interval_labels``).

Network (all FP64 here):
    x   = [o (3), d (3), code (6 J)]       ray origin, unit direction, pose code
    z1  = W1 x + b1,   h1 = relu(z1)        W1: [64][6 + 6J]
    z2  = W2 h1 + b2,  h2 = relu(z2)        W2: [64][64]
    z3  = W3 h2 + b3,  h3 = relu(z3)        W3: [64][64]
    z4  = W4 h3 + b4,  y  = sigmoid(z4)     W4: [2][64];  y = (u_near, u_far)
The pose code of a pose is, for every bone j, the first two columns of its
local rotation Rot(r_j) (the 6-D rotation representation), column by column.
Loss: mean over rays and both outputs of SmoothL1 with beta = 1 (default), or
the one-sided form: on rays whose label holds a sample (u_near <= u_far) the
pinball (quantile) loss rho_tau(t - y) = max(tau (t - y), (tau - 1) (t - y))
with a level tau per output - its minimiser over a constant is the
tau-quantile of the targets, so a small tau for u_near makes late starts rare
and a large one for u_far early ends - and SmoothL1 on rays with the empty
label (1, 0), which keeps them predicted empty (a quantile of an empty
interval has no meaning).
Training: Adam with bias correction.

Flat parameter order (FP32 on the GPU, the same order here):
    W1 (row-major), b1, W2, b2, W3, b3, W4, b4.

``precision`` selects how the matrix products are rounded (everything else
stays FP64):
  "fp64"   - plain FP64 (the definition);
  "bf16"   - both operands of every product rounded to bfloat16 before an
             FP64 product: the network's inference form (BF16 matrix-core
             operands, wide accumulation);
  "bf16x3" - every operand split into a bfloat16 head and a bfloat16 tail
             (a = a_hi + a_lo, a_lo = bf16(a - a_hi)) and the product taken
             as a_hi b_hi + a_hi b_lo + a_lo b_hi: the training form (three
             BF16 matrix-core products per product, about 16 significant bits).
In the "bf16" forms the pose-code part of the first layer, W1[:, 6:] code +
b1, depends only on the pose and is evaluated once per pose at full
precision (it enters every ray of the pose as a bias), and the bias
gradients are plain sums of the deltas.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from . import bf16_round, rodrigues

HIDDEN = 64


def input_dim(J: int) -> int:
    return 6 + 6 * J


def param_shapes(J: int) -> List[Tuple[str, Tuple[int, ...]]]:
    n_in = input_dim(J)
    return [("W1", (HIDDEN, n_in)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
            ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,)), ("W4", (2, HIDDEN)), ("b4", (2,))]


def param_count(J: int) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(J))


def unpack(theta: np.ndarray, J: int) -> Dict[str, np.ndarray]:
    theta = np.asarray(theta, dtype=np.float64).reshape(-1)
    assert theta.size == param_count(J)
    out, k = {}, 0
    for name, shp in param_shapes(J):
        m = int(np.prod(shp))
        out[name] = theta[k:k + m].reshape(shp)
        k += m
    return out


def pack(p: Dict[str, np.ndarray], J: int) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in param_shapes(J)])


def pose_code(r: np.ndarray) -> np.ndarray:
    """[P][J][3] axis-angle local rotations -> [P][6J]: per bone the first and
    second column of Rot(r_j)."""
    r = np.asarray(r, dtype=np.float64)
    P, J, _ = r.shape
    out = np.zeros((P, 6 * J))
    for p in range(P):
        for j in range(J):
            R = rodrigues(r[p, j])
            out[p, 6 * j:6 * j + 3] = R[:, 0]
            out[p, 6 * j + 3:6 * j + 6] = R[:, 1]
    return out


def inputs(o: np.ndarray, d: np.ndarray, code: np.ndarray) -> np.ndarray:
    """Rows [o, d, code] of the network input for rays (o, d) of one pose."""
    o = np.asarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
    code = np.broadcast_to(np.asarray(code, dtype=np.float64), (o.shape[0], code.shape[-1]))
    return np.concatenate([o, d, code], axis=1)


PRECISIONS = ("fp64", "bf16", "bf16x3")


def _bf(x: np.ndarray) -> np.ndarray:
    return bf16_round(x).astype(np.float64)


def _mm(a: np.ndarray, b: np.ndarray, precision: str) -> np.ndarray:
    """a @ b with the operand rounding of `precision`."""
    if precision == "fp64":
        return a @ b
    if precision == "bf16":
        return _bf(a) @ _bf(b)
    if precision == "bf16x3":
        ah = _bf(a)
        bh = _bf(b)
        al = _bf(a - ah)
        bl = _bf(b - bh)
        return al @ bh + ah @ bl + ah @ bh
    raise ValueError(precision)


def sigmoid(z: np.ndarray) -> np.ndarray:
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(theta: np.ndarray, X: np.ndarray, J: int, precision: str = "fp64"):
    """Outputs y [n][2] and the activations of every layer."""
    p = unpack(theta, J)
    X = np.asarray(X, dtype=np.float64)
    z1 = _mm(X[:, :6], p["W1"][:, :6].T, precision) + (X[:, 6:] @ p["W1"][:, 6:].T + p["b1"])
    h1 = np.maximum(z1, 0.0)
    z2 = _mm(h1, p["W2"].T, precision) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = _mm(h2, p["W3"].T, precision) + p["b3"]
    h3 = np.maximum(z3, 0.0)
    z4 = _mm(h3, p["W4"].T, precision) + p["b4"]
    y = sigmoid(z4)
    return y, {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "z3": z3, "h3": h3, "z4": z4, "y": y}


def smooth_l1(e: np.ndarray, beta: float = 1.0) -> np.ndarray:
    """Elementwise SmoothL1: e^2 / (2 beta) where |e| < beta, else |e| - beta / 2."""
    a = np.abs(e)
    return np.where(a < beta, 0.5 * e * e / beta, a - 0.5 * beta)


def smooth_l1_grad(e: np.ndarray, beta: float = 1.0) -> np.ndarray:
    return np.where(np.abs(e) < beta, e / beta, np.sign(e))


def pinball(r: np.ndarray, tau) -> np.ndarray:
    """Elementwise pinball loss of the residual r = target - prediction at level
    tau (broadcast over the last axis): tau r for r >= 0, (tau - 1) r below."""
    tau = np.asarray(tau, dtype=np.float64)
    return np.maximum(tau * r, (tau - 1.0) * r)


def pinball_grad(r: np.ndarray, tau) -> np.ndarray:
    """d pinball / d prediction: -tau where the target is above the prediction,
    1 - tau where it is below, 0 where they are equal."""
    tau = np.asarray(tau, dtype=np.float64) * np.ones_like(r)
    return np.where(r > 0, -tau, np.where(r < 0, 1.0 - tau, 0.0))


def _hit_rows(t: np.ndarray) -> np.ndarray:
    """Rays whose label holds a sample (u_near <= u_far), as a column mask."""
    return (t[:, 0] <= t[:, 1])[:, None]


def loss(y: np.ndarray, target: np.ndarray, kind: str = "smooth_l1", tau=(0.5, 0.5)) -> float:
    """Mean over rays and both outputs of SmoothL1 (beta = 1), or of the
    one-sided form: pinball at levels tau = (tau_near, tau_far) on rays with
    a sample, SmoothL1 on rays with the empty label."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    if kind == "pinball":
        return float(np.where(_hit_rows(t), pinball(t - y, tau), smooth_l1(y - t)).mean())
    return float(smooth_l1(y - t).mean())


def grad(theta: np.ndarray, X: np.ndarray, target: np.ndarray, J: int,
         precision: str = "fp64", kind: str = "smooth_l1", tau=(0.5, 0.5)) -> Tuple[float, np.ndarray]:
    """Loss (`kind`, levels `tau` for the pinball loss) and its gradient with
    respect to the flat parameters, by the chain rule written out layer by
    layer (backpropagation)."""
    p = unpack(theta, J)
    y, a = forward(theta, X, J, precision)
    t = np.asarray(target, dtype=np.float64)
    n = y.shape[0]
    L = loss(y, t, kind, tau)
    if kind == "pinball":
        dy = np.where(_hit_rows(t), pinball_grad(t - y, tau), smooth_l1_grad(y - t)) / (2.0 * n)   # dL/dy
    else:
        dy = smooth_l1_grad(y - t) / (2.0 * n)      # dL/dy
    d4 = dy * y * (1.0 - y)                          # dL/dz4 (sigmoid')
    g = {"W4": _mm(d4.T, a["h3"], precision), "b4": d4.sum(axis=0)}
    d3 = _mm(d4, p["W4"], precision) * (a["z3"] > 0)
    g["W3"] = _mm(d3.T, a["h2"], precision)
    g["b3"] = d3.sum(axis=0)
    d2 = _mm(d3, p["W3"], precision) * (a["z2"] > 0)
    g["W2"] = _mm(d2.T, a["h1"], precision)
    g["b2"] = d2.sum(axis=0)
    d1 = _mm(d2, p["W2"], precision) * (a["z1"] > 0)
    g["W1"] = _mm(d1.T, a["X"], precision)
    g["b1"] = d1.sum(axis=0)
    return L, pack(g, J)


def adam_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, step: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1): moments, bias correction, update.
    Returns the new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    theta = theta - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v


_M64 = (1 << 64) - 1


def splitmix64(seed: int, k: int) -> int:
    """Output k (k = 1, 2, ...) of the SplitMix64 stream of `seed` (Steele, Lea
    and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
    the state after k steps of the odd increment 0x9E3779B97F4A7C15, mixed by
    two xor-shift-multiply rounds and a final xor-shift (64-bit arithmetic)."""
    z = (seed + k * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def init_params(J: int, seed: int) -> np.ndarray:
    """Seeded initial parameters (flat order, float32): parameter i of a layer
    with fan-in m is (2u - 1) / sqrt(m), u = (top 24 bits of output i + 1 of
    the SplitMix64 stream of `seed`) / 2^24, so every value lies in
    (-1/sqrt(m), 1/sqrt(m)) - the uniform initialisation of fully connected
    layers."""
    out = np.empty(param_count(J), dtype=np.float32)
    i = 0
    for name, shape in param_shapes(J):
        fan_in = input_dim(J) if name in ("W1", "b1") else HIDDEN
        k = 1.0 / math.sqrt(fan_in)
        for _ in range(int(np.prod(shape))):
            u = (splitmix64(seed, i + 1) >> 40) * 2.0 ** -24
            out[i] = np.float32((2.0 * u - 1.0) * k)
            i += 1
    return out
