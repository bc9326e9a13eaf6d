// The shading network's last 3x3 convolution with its 1x1 head fused (the
// network's output layer of Section 3.1 / Section 6 "Light" variant).
#pragma once
#include "internal.h"

namespace art {

// out_k = sigmoid(b[k] + sum_c w[k][c] x_c) over the convolution's 32 output
// channels x (after bias and ReLU, rounded to FP16 as a stored activation is),
// written planar [N][4][H][W] in FP32.
struct ConvHead {
    const float* w;   // [4][32]
    const float* b;   // [4]
    float* out;
};

// The convolution `a` (Cout = 32) followed by the head: `a.out` is not written.
hipError_t launch_conv3x3_head(const ConvLaunch& a, const ConvHead& h, hipStream_t st);

}  // namespace art
