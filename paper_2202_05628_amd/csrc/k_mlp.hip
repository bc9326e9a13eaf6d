// Learned ray-interval proposal network on the matrix cores (an addition to
// the paper's renderer; the quantity it predicts is defined by the renderer's
// composited samples, Section 3.1, Eq. 5-6).
//
// Network: x = [o (3), d (3), pose code (6J)] -> 64 -> 64 -> 64 (ReLU) -> 2
// (sigmoid) = (u_near, u_far).  The pose-code part of the first layer,
// c_p = W1[:, 6:] code_p + b1, depends only on the pose and is evaluated once
// per pose in FP32 (k_mlp_prep); per ray the first layer is the 6-input
// product plus that bias.  Every other product runs on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation and FP32 master weights:
// inference takes single BF16 operands; training splits every operand into a
// BF16 head and tail (a = a_hi + a_lo) and takes a_hi b_hi + a_hi b_lo +
// a_lo b_hi (three matrix-core products, about 16 significant bits), so the
// gradients are not dominated by operand rounding.
//
// Register layout of one wave working on 16 rays (lane l, r = l % 16,
// g = l / 16):
//   accumulator tile t (f32x4): lane holds h[ray r][16 t + 4 g + e], e < 4;
//   B operand of k-step ks (8 x bf16): lane holds h[ray r][phi(ks, g, e)],
//     phi(ks, g, e) = 16 (2 ks + e / 4) + 4 g + e % 4, e < 8,
//   i.e. the accumulators of tiles 2 ks and 2 ks + 1 - a layer's output feeds
//   the next layer without moving data between lanes; the weight operands are
//   packed with the same feature permutation over K (k_mlp_prep);
//   A operand (weights): lane holds W[16 m + r][phi(ks, g, e)].
// The weight gradients are contractions over rays: the training forward /
// backward kernel stores activations and deltas (FP32) feature-major, and
// k_mlp_wgrad reads 8 consecutive rays per lane as the K operand.  Partial
// sums per chunk of 256 rays are reduced in a fixed order (deterministic).
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace art {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHid = 64;
// packed operand blocks (64 lanes x 8 bf16 each)
constexpr int kB_W1 = 0;     // [mt]      first layer, 6 inputs padded to K = 32
constexpr int kB_W2 = 4;     // [mt][ks]
constexpr int kB_W3 = 12;    // [mt][ks]
constexpr int kB_W4 = 20;    // [ks]      2 outputs padded to 16 rows
constexpr int kB_W4T = 22;   // [mt]      W4^T, K = 2 outputs padded to 32
constexpr int kB_W3T = 26;   // [mt][ks]
constexpr int kB_W2T = 34;   // [mt][ks]
constexpr int kBlocks = 42;
constexpr int kPacked = 2 * kBlocks * 64 * 8;   // heads, then tails
// feature-major training scratch rows
constexpr int kRowH1 = 0, kRowH2 = 64, kRowH3 = 128, kRowD1 = 192, kRowD2 = 256, kRowD3 = 320, kRowD4 = 384;
constexpr int kRows = 400;
constexpr int kChunk = 256;   // rays per weight-gradient partial

__device__ inline uint16_t f2bf(float x) {   // round to nearest even
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline bf16x8 pack8(float v0, float v1, float v2, float v3, float v4, float v5, float v6, float v7) {
    u16x8 u;
    u[0] = f2bf(v0);
    u[1] = f2bf(v1);
    u[2] = f2bf(v2);
    u[3] = f2bf(v3);
    u[4] = f2bf(v4);
    u[5] = f2bf(v5);
    u[6] = f2bf(v6);
    u[7] = f2bf(v7);
    return __builtin_bit_cast(bf16x8, u);
}

__device__ inline bf16x8 pack_tiles(const f32x4 a, const f32x4 b) {
    return pack8(a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]);
}

__device__ inline f32x4 mfma(const bf16x8 a, const bf16x8 b, const f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// v = hi + lo with hi = bf16(v), lo = bf16(v - hi)
__device__ inline void split8(const float* v, bf16x8& hi, bf16x8& lo) {
    u16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = f2bf(v[e]);
        l[e] = f2bf(v[e] - __uint_as_float((uint32_t)h[e] << 16));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

// B operands (head, tail) of the two k-steps of a 64-wide layer input held
// as four accumulator tiles.
template <bool SPLIT>
__device__ inline void tiles_to_ops(const f32x4* t, bf16x8* Bh, bf16x8* Bl) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const float v[8] = {t[2 * ks][0], t[2 * ks][1], t[2 * ks][2], t[2 * ks][3],
                            t[2 * ks + 1][0], t[2 * ks + 1][1], t[2 * ks + 1][2], t[2 * ks + 1][3]};
        if (SPLIT) split8(v, Bh[ks], Bl[ks]);
        else Bh[ks] = pack8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
    }
}

// A [16 x K] x B [K x 16] with K = 32 (one k-step): one or three products.
template <bool SPLIT, typename WSrc>
__device__ inline f32x4 mm1(const WSrc& w, int blk, const bf16x8 Bh, const bf16x8 Bl, f32x4 acc) {
    if (SPLIT) {
        acc = mfma(w.lo(blk), Bh, acc);
        acc = mfma(w.get(blk), Bl, acc);
    }
    return mfma(w.get(blk), Bh, acc);
}

__host__ __device__ inline int phi(int ks, int g, int e) { return 16 * (2 * ks + (e >> 2)) + 4 * g + (e & 3); }

__device__ inline float sigmoidf(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Ray of pixel (px, py) of a camera in FP32 (network input only).
__device__ inline void ray_f32(const CamParams& cam, int px, int py, float* o, float* d) {
    const float dcx = ((float)px + 0.5f - (float)cam.cx) / (float)cam.fx;
    const float dcy = ((float)py + 0.5f - (float)cam.cy) / (float)cam.fy;
    float n2 = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] = (float)cam.R[3 * i] * dcx + (float)cam.R[3 * i + 1] * dcy + (float)cam.R[3 * i + 2];
        n2 += d[i] * d[i];
    }
    const float inv = 1.0f / sqrtf(n2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] *= inv;
        o[i] = (float)cam.t[i];
    }
}

// ---------------------------------------------------------------------------
// pose code: per pose and bone the first two columns of Rot(r_j)
// ---------------------------------------------------------------------------
__global__ void k_pose_code(const double* __restrict__ pose, int J, int P, float* __restrict__ code) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * J) return;
    const int p = i / J, j = i % J;
    double M[9];
    axis_angle_to_matrix(pose + ((size_t)p * (J + 2) + j) * 3, M);
    float* c = code + (size_t)p * 6 * J + 6 * j;
    c[0] = (float)M[0];
    c[1] = (float)M[3];
    c[2] = (float)M[6];
    c[3] = (float)M[1];
    c[4] = (float)M[4];
    c[5] = (float)M[7];
}

// ---------------------------------------------------------------------------
// operand packing + per-pose first-layer bias
// ---------------------------------------------------------------------------
__global__ void k_mlp_prep(const float* __restrict__ theta, MlpDims m, const float* __restrict__ code, int P,
                           uint16_t* __restrict__ packed, float* __restrict__ cbias) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float* W1 = theta + m.oW1;
    const float* W2 = theta + m.oW2;
    const float* W3 = theta + m.oW3;
    const float* W4 = theta + m.oW4;
    if (i < kPacked) {
        const int half = kPacked / 2;
        const bool tail = i >= half;
        const int ii = tail ? i - half : i;
        const int blk = ii / 512, lane = (ii / 8) % 64, e = ii % 8;
        const int r = lane & 15, g = lane >> 4;
        float v = 0.0f;
        if (blk < kB_W2) {
            const int mt = blk - kB_W1, k = 8 * g + e;
            v = k < 6 ? W1[(16 * mt + r) * m.n_in + k] : 0.0f;
        } else if (blk < kB_W3) {
            const int mt = (blk - kB_W2) >> 1, ks = (blk - kB_W2) & 1;
            v = W2[(16 * mt + r) * kHid + phi(ks, g, e)];
        } else if (blk < kB_W4) {
            const int mt = (blk - kB_W3) >> 1, ks = (blk - kB_W3) & 1;
            v = W3[(16 * mt + r) * kHid + phi(ks, g, e)];
        } else if (blk < kB_W4T) {
            const int ks = blk - kB_W4;
            v = r < 2 ? W4[r * kHid + phi(ks, g, e)] : 0.0f;
        } else if (blk < kB_W3T) {
            const int mt = blk - kB_W4T, k = 8 * g + e;
            v = k < 2 ? W4[k * kHid + 16 * mt + r] : 0.0f;
        } else if (blk < kB_W2T) {
            const int mt = (blk - kB_W3T) >> 1, ks = (blk - kB_W3T) & 1;
            v = W3[phi(ks, g, e) * kHid + 16 * mt + r];
        } else {
            const int mt = (blk - kB_W2T) >> 1, ks = (blk - kB_W2T) & 1;
            v = W2[phi(ks, g, e) * kHid + 16 * mt + r];
        }
        const uint16_t hb = f2bf(v);
        packed[i] = tail ? f2bf(v - __uint_as_float((uint32_t)hb << 16)) : hb;
        return;
    }
    const int j = i - kPacked;
    if (j >= P * kHid) return;
    const int p = j / kHid, o = j % kHid;
    const int nc = m.n_in - 6;
    const float* w = W1 + (size_t)o * m.n_in + 6;
    const float* c = code + (size_t)p * nc;
    float s = theta[m.ob1 + o];
    for (int k = 0; k < nc; ++k) s = __fmaf_rn(w[k], c[k], s);
    cbias[j] = s;
}

// Layer 2..4 forward of one 16-ray group from the layer-1 output h1.
template <bool SPLIT, typename WSrc>
__device__ inline void forward_tail(const WSrc& w, const float* __restrict__ theta, const MlpDims& m, int g,
                                    const f32x4* h1, f32x4* h2, f32x4* h3, f32x4& z4) {
    bf16x8 Bh[2], Bl[2];
    tiles_to_ops<SPLIT>(h1, Bh, Bl);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mm1<SPLIT>(w, kB_W2 + 2 * mt, Bh[0], Bl[0], acc);
        acc = mm1<SPLIT>(w, kB_W2 + 2 * mt + 1, Bh[1], Bl[1], acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fmaxf(acc[e] + theta[m.ob2 + 16 * mt + 4 * g + e], 0.0f);
        h2[mt] = acc;
    }
    tiles_to_ops<SPLIT>(h2, Bh, Bl);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mm1<SPLIT>(w, kB_W3 + 2 * mt, Bh[0], Bl[0], acc);
        acc = mm1<SPLIT>(w, kB_W3 + 2 * mt + 1, Bh[1], Bl[1], acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fmaxf(acc[e] + theta[m.ob3 + 16 * mt + 4 * g + e], 0.0f);
        h3[mt] = acc;
    }
    tiles_to_ops<SPLIT>(h3, Bh, Bl);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mm1<SPLIT>(w, kB_W4, Bh[0], Bl[0], acc);
    acc = mm1<SPLIT>(w, kB_W4 + 1, Bh[1], Bl[1], acc);
    z4 = acc;
}

// First layer: 6 ray inputs (lanes of group 0 carry them) plus the pose bias.
template <bool SPLIT, typename WSrc>
__device__ inline void forward_head(const WSrc& w, const float* x, const float* __restrict__ cb, int g, f32x4* h1) {
    const float v[8] = {g == 0 ? x[0] : 0.0f, g == 0 ? x[1] : 0.0f, g == 0 ? x[2] : 0.0f, g == 0 ? x[3] : 0.0f,
                        g == 0 ? x[4] : 0.0f, g == 0 ? x[5] : 0.0f, 0.0f, 0.0f};
    bf16x8 Bh, Bl;
    if (SPLIT) split8(v, Bh, Bl);
    else Bh = pack8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mm1<SPLIT>(w, kB_W1 + mt, Bh, Bl, acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fmaxf(acc[e] + cb[16 * mt + 4 * g + e], 0.0f);
        h1[mt] = acc;
    }
}

struct WGlobal {   // operand blocks read from device memory (heads, tails)
    const bf16x8* p;
    int lane;
    __device__ bf16x8 get(int blk) const { return p[blk * 64 + lane]; }
    __device__ bf16x8 lo(int blk) const { return p[(kBlocks + blk) * 64 + lane]; }
};

struct WRegs {   // forward operand heads held in registers (inference)
    bf16x8 b[kB_W4T];
    __device__ bf16x8 get(int blk) const { return b[blk]; }
    __device__ bf16x8 lo(int blk) const { return b[blk]; }   // unused: single BF16 operands
};

// ---------------------------------------------------------------------------
// inference precision (single BF16 operands): the biases enter as the
// accumulator input of a layer's first product, activations are rounded to
// BF16 by the hardware conversion (round to nearest even, as f2bf) and the
// ReLU is taken on the rounded values (rounding keeps the sign, so this is
// the ReLU of the FP32 value, rounded), as a 16-bit integer maximum with 0.
// ---------------------------------------------------------------------------
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t cvt2(float a, float b) {   // two floats -> packed BF16 (a in the low half)
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ inline uint32_t relu2(uint32_t h) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), s16x2{0, 0}));
}
__device__ inline bf16x8 cvt8(float v0, float v1, float v2, float v3, float v4, float v5, float v6, float v7) {
    return __builtin_bit_cast(bf16x8, u32x4{cvt2(v0, v1), cvt2(v2, v3), cvt2(v4, v5), cvt2(v6, v7)});
}
__device__ inline bf16x8 relu_bf16(const f32x4 a, const f32x4 b) {
    return __builtin_bit_cast(bf16x8, u32x4{relu2(cvt2(a[0], a[1])), relu2(cvt2(a[2], a[3])),
                                            relu2(cvt2(b[0], b[1])), relu2(cvt2(b[2], b[3]))});
}

// Per-lane layer biases in accumulator layout (element e of tile mt is
// output 16 mt + 4 g + e).
struct InferBias {
    f32x4 b2[4], b3[4];
    float b4[2];
};
__device__ inline void load_infer_bias(const float* __restrict__ theta, const MlpDims& m, int g, InferBias& B) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            B.b2[mt][e] = theta[m.ob2 + 16 * mt + 4 * g + e];
            B.b3[mt][e] = theta[m.ob3 + 16 * mt + 4 * g + e];
        }
    B.b4[0] = theta[m.ob4];
    B.b4[1] = theta[m.ob4 + 1];
}
__device__ inline void load_pose_bias(const float* __restrict__ cb, int g, f32x4* c1) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) c1[mt][e] = cb[16 * mt + 4 * g + e];
}

// Outputs (u_near, u_far) of the 16 rays of a group; x: the ray inputs, read
// by the lanes of group 0 (g = 0) only; c1: the pose's first-layer bias.
template <typename WSrc>
__device__ inline float2 infer_group(const WSrc& w, const InferBias& B, const f32x4* c1, const float* x, int g) {
    const bf16x8 X = cvt8(g == 0 ? x[0] : 0.0f, g == 0 ? x[1] : 0.0f, g == 0 ? x[2] : 0.0f, g == 0 ? x[3] : 0.0f,
                          g == 0 ? x[4] : 0.0f, g == 0 ? x[5] : 0.0f, 0.0f, 0.0f);
    f32x4 t[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) t[mt] = mfma(w.get(kB_W1 + mt), X, c1[mt]);
    bf16x8 H0 = relu_bf16(t[0], t[1]), H1 = relu_bf16(t[2], t[3]);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) t[mt] = mfma(w.get(kB_W2 + 2 * mt + 1), H1, mfma(w.get(kB_W2 + 2 * mt), H0, B.b2[mt]));
    H0 = relu_bf16(t[0], t[1]);
    H1 = relu_bf16(t[2], t[3]);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) t[mt] = mfma(w.get(kB_W3 + 2 * mt + 1), H1, mfma(w.get(kB_W3 + 2 * mt), H0, B.b3[mt]));
    H0 = relu_bf16(t[0], t[1]);
    H1 = relu_bf16(t[2], t[3]);
    const f32x4 z = mfma(w.get(kB_W4 + 1), H1, mfma(w.get(kB_W4), H0, f32x4{B.b4[0], B.b4[1], 0.0f, 0.0f}));
    // sigmoid with the hardware reciprocal (1 ulp)
    return make_float2(__builtin_amdgcn_rcpf(1.0f + __expf(-z[0])), __builtin_amdgcn_rcpf(1.0f + __expf(-z[1])));
}

// ---------------------------------------------------------------------------
// forward (mode 0) / forward + loss + backward (mode 1) over n rays
// ---------------------------------------------------------------------------
struct FbArgs {
    const uint16_t* packed;
    const float* theta;
    const float* cbias;       // [P][64]
    MlpDims m;
    const float* od;          // [n][6]
    const int32_t* pose;      // [n]
    const float* target;      // [n][2]
    float* out;               // [n][2] (mode 0)
    int64_t n, n_pad;         // n_pad: multiple of kChunk
    float* S;                 // [kRows][n_pad] (mode 1)
    float* loss_part;         // [gridDim.x] sums of the loss over rays and outputs
    float inv2n;              // 1 / (2 n)
    MlpLoss loss;             // SmoothL1 or pinball (levels per output)
    int mode;
    int P;                    // valid pose ids: 0..P-1
    uint32_t* bad;            // set to 1 when a pose id is out of range
};

__device__ inline float smooth_l1f(float e) { const float a = fabsf(e); return a < 1.0f ? 0.5f * e * e : a - 0.5f; }
__device__ inline float smooth_l1_gradf(float e) { return fabsf(e) < 1.0f ? e : (e > 0.0f ? 1.0f : -1.0f); }
// pinball loss of the error e = prediction - target at level tau, and its
// derivative with respect to the prediction
__device__ inline float pinballf(float e, float tau) { return e > 0.0f ? (1.0f - tau) * e : -tau * e; }
__device__ inline float pinball_gradf(float e, float tau) { return e > 0.0f ? 1.0f - tau : (e < 0.0f ? -tau : 0.0f); }

__device__ inline void store_tiles(float* S, int64_t stride, int row0, int64_t ray, int g, const f32x4* t, int nt) {
    for (int mt = 0; mt < nt; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) S[(int64_t)(row0 + 16 * mt + 4 * g + e) * stride + ray] = t[mt][e];
}

template <bool SPLIT>
__device__ inline void fb_body(const FbArgs& a, int lane, int w, float* sloss) {
    const int r = lane & 15, g = lane >> 4;
    WGlobal W{reinterpret_cast<const bf16x8*>(a.packed), lane};
    const MlpDims& m = a.m;
    float lsum = 0.0f;
    const int64_t groups = a.n_pad / 16;
    for (int64_t grp = (int64_t)blockIdx.x * 4 + w; grp < groups; grp += (int64_t)gridDim.x * 4) {
        const int64_t ray = grp * 16 + r;
        bool valid = ray < a.n;
        float x[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        int p = 0;
        if (valid) {
            p = a.pose[ray];
            if ((unsigned)p >= (unsigned)a.P) {   // a ray with a bad pose id is left out
                atomicOr(a.bad, 1u);
                valid = false;
                p = 0;
            }
        }
        if (valid) {
#pragma unroll
            for (int i = 0; i < 6; ++i) x[i] = a.od[ray * 6 + i];
        }
        if constexpr (!SPLIT) {
            InferBias B;
            load_infer_bias(a.theta, m, g, B);
            f32x4 c1[4];
            load_pose_bias(a.cbias + (size_t)p * kHid, g, c1);
            const float2 y = infer_group(W, B, c1, x, g);
            if (valid && g == 0) reinterpret_cast<float2*>(a.out)[ray] = y;
            continue;
        }
        f32x4 h1[4], h2[4], h3[4], z4;
        forward_head<SPLIT>(W, x, a.cbias + (size_t)p * kHid, g, h1);
        forward_tail<SPLIT>(W, a.theta, m, g, h1, h2, h3, z4);
        const float y0 = sigmoidf(z4[0] + a.theta[m.ob4]);
        const float y1 = sigmoidf(z4[1] + a.theta[m.ob4 + 1]);
        // loss and dL/dz4 (lanes of group 0 hold the two outputs of ray r)
        float d40 = 0.0f, d41 = 0.0f;
        if (valid && g == 0) {
            const float t0 = a.target[ray * 2], t1 = a.target[ray * 2 + 1];
            const float e0 = y0 - t0, e1 = y1 - t1;
            float g0, g1;
            if (a.loss.kind == 1 && t0 <= t1) {   // one-sided form: pinball on rays with a sample
                lsum += pinballf(e0, a.loss.tau[0]) + pinballf(e1, a.loss.tau[1]);
                g0 = pinball_gradf(e0, a.loss.tau[0]);
                g1 = pinball_gradf(e1, a.loss.tau[1]);
            } else {
                lsum += smooth_l1f(e0) + smooth_l1f(e1);
                g0 = smooth_l1_gradf(e0);
                g1 = smooth_l1_gradf(e1);
            }
            d40 = g0 * a.inv2n * y0 * (1.0f - y0);
            d41 = g1 * a.inv2n * y1 * (1.0f - y1);
        }
        store_tiles(a.S, a.n_pad, kRowH1, ray, g, h1, 4);
        store_tiles(a.S, a.n_pad, kRowH2, ray, g, h2, 4);
        store_tiles(a.S, a.n_pad, kRowH3, ray, g, h3, 4);
        {
            const f32x4 d4 = {d40, d41, 0.0f, 0.0f};   // zero for g > 0
            store_tiles(a.S, a.n_pad, kRowD4, ray, g, &d4, 1);
        }
        bf16x8 Bh[2], Bl[2];
        {
            const float v[8] = {d40, d41, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            split8(v, Bh[0], Bl[0]);
        }
        f32x4 d3[4], d2[4], d1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mm1<true>(W, kB_W4T + mt, Bh[0], Bl[0], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = h3[mt][e] > 0.0f ? acc[e] : 0.0f;
            d3[mt] = acc;
        }
        store_tiles(a.S, a.n_pad, kRowD3, ray, g, d3, 4);
        tiles_to_ops<true>(d3, Bh, Bl);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mm1<true>(W, kB_W3T + 2 * mt, Bh[0], Bl[0], acc);
            acc = mm1<true>(W, kB_W3T + 2 * mt + 1, Bh[1], Bl[1], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = h2[mt][e] > 0.0f ? acc[e] : 0.0f;
            d2[mt] = acc;
        }
        store_tiles(a.S, a.n_pad, kRowD2, ray, g, d2, 4);
        tiles_to_ops<true>(d2, Bh, Bl);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mm1<true>(W, kB_W2T + 2 * mt, Bh[0], Bl[0], acc);
            acc = mm1<true>(W, kB_W2T + 2 * mt + 1, Bh[1], Bl[1], acc);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = h1[mt][e] > 0.0f ? acc[e] : 0.0f;
            d1[mt] = acc;
        }
        store_tiles(a.S, a.n_pad, kRowD1, ray, g, d1, 4);
    }
    if (!SPLIT) return;
    lsum = wave_sum(lsum);
    if (lane == 0) sloss[w] = lsum;
}

// mode 0: network outputs (inference precision, single BF16 operands);
// mode 1: training forward + loss + backward (split BF16 operands).
__global__ __launch_bounds__(256) void k_mlp_fb(FbArgs a) {
    __shared__ float sloss[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (a.mode == 0) {
        fb_body<false>(a, lane, w, sloss);
        return;
    }
    fb_body<true>(a, lane, w, sloss);
    __syncthreads();
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = ((sloss[0] + sloss[1]) + sloss[2]) + sloss[3];
}

// ---------------------------------------------------------------------------
// weight gradients of one chunk of 256 rays: dW = sum_rays delta (x) input
// ---------------------------------------------------------------------------
struct WgArgs {
    const float* S;
    int64_t n, n_pad;
    const float* od;
    const int32_t* pose;
    const float* code;     // [P][6J]
    int P;
    MlpDims m;
    float* part;           // [n_pad / kChunk][np]
};

__device__ inline void load8_split(const float* p, bf16x8& hi, bf16x8& lo) {
    const float4 a = reinterpret_cast<const float4*>(p)[0];
    const float4 b = reinterpret_cast<const float4*>(p)[1];
    const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    split8(v, hi, lo);
}

__global__ __launch_bounds__(256) void k_mlp_wgrad(WgArgs a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const MlpDims& m = a.m;
    const int64_t R0 = (int64_t)blockIdx.x * kChunk;
    float* part = a.part + (size_t)blockIdx.x * m.np;
    const int nt1 = (m.n_in + 15) / 16;
    const int ntiles = 4 * nt1 + 16 + 16 + 4;
    const int nc = m.n_in - 6;
    for (int t = w; t < ntiles; t += 4) {
        int layer, mt, nt;
        if (t < 4 * nt1) {
            layer = 1;
            mt = t / nt1;
            nt = t % nt1;
        } else if (t < 4 * nt1 + 16) {
            layer = 2;
            mt = (t - 4 * nt1) / 4;
            nt = (t - 4 * nt1) % 4;
        } else if (t < 4 * nt1 + 32) {
            layer = 3;
            mt = (t - 4 * nt1 - 16) / 4;
            nt = (t - 4 * nt1 - 16) % 4;
        } else {
            layer = 4;
            mt = 0;
            nt = t - 4 * nt1 - 32;
        }
        const int arow = layer == 1 ? kRowD1 + 16 * mt + r
                       : layer == 2 ? kRowD2 + 16 * mt + r
                       : layer == 3 ? kRowD3 + 16 * mt + r
                                    : kRowD4 + r;
        const int brow = layer == 2 ? kRowH1 : layer == 3 ? kRowH2 : kRowH3;
        const int in = 16 * nt + r;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int kb = 0; kb < kChunk / 32; ++kb) {
            const int64_t rb = R0 + kb * 32 + 8 * g;
            bf16x8 Ah, Al, Bh, Bl;
            load8_split(a.S + (int64_t)arow * a.n_pad + rb, Ah, Al);
            if (layer == 1) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int64_t ray = rb + e;
                    float x = 0.0f;
                    if (ray < a.n) {
                        const int p = a.pose[ray];
                        if ((unsigned)p < (unsigned)a.P) {
                            if (in < 6) x = a.od[ray * 6 + in];
                            else if (in < m.n_in) x = a.code[(size_t)p * nc + (in - 6)];
                        }
                    }
                    v[e] = x;
                }
                split8(v, Bh, Bl);
            } else {
                load8_split(a.S + (int64_t)(brow + in) * a.n_pad + rb, Bh, Bl);
            }
            acc = mfma(Al, Bh, acc);
            acc = mfma(Ah, Bl, acc);
            acc = mfma(Ah, Bh, acc);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int out = 16 * mt + 4 * g + e;
            if (layer == 1) {
                if (in < m.n_in) part[m.oW1 + (size_t)out * m.n_in + in] = acc[e];
            } else if (layer == 2) {
                part[m.oW2 + out * kHid + in] = acc[e];
            } else if (layer == 3) {
                part[m.oW3 + out * kHid + in] = acc[e];
            } else if (out < 2) {
                part[m.oW4 + out * kHid + in] = acc[e];
            }
        }
    }
    // bias gradients: sums of the stored deltas
    for (int row = threadIdx.x; row < 3 * kHid + 2; row += blockDim.x) {
        int srow, dst;
        if (row < kHid) { srow = kRowD1 + row; dst = m.ob1 + row; }
        else if (row < 2 * kHid) { srow = kRowD2 + row - kHid; dst = m.ob2 + row - kHid; }
        else if (row < 3 * kHid) { srow = kRowD3 + row - 2 * kHid; dst = m.ob3 + row - 2 * kHid; }
        else { srow = kRowD4 + row - 3 * kHid; dst = m.ob4 + row - 3 * kHid; }
        const float* s = a.S + (int64_t)srow * a.n_pad + R0;
        float acc = 0.0f;
        for (int i = 0; i < kChunk; ++i) acc += s[i];
        part[dst] = acc;
    }
}

// ---------------------------------------------------------------------------
// fixed-order reduction of the partials (+ Adam) and of the loss
// ---------------------------------------------------------------------------
struct RedArgs {
    const float* part;
    int nchunks;
    int np;
    float* grad;           // may be null
    float* theta;
    float* m1;
    float* m2;
    int adam;
    float lr, beta1, beta2, eps, bc1, bc2;
    const float* loss_part;
    int nloss;
    float inv2n;
    float* loss_out;       // may be null
};

__global__ __launch_bounds__(256) void k_mlp_reduce(RedArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && a.loss_out) {
        float L = 0.0f;
        for (int k = 0; k < a.nloss; ++k) L += a.loss_part[k];
        *a.loss_out = L * a.inv2n;
    }
    if (i >= a.np) return;
    float gsum = 0.0f;
    for (int c = 0; c < a.nchunks; ++c) gsum += a.part[(size_t)c * a.np + i];
    if (a.grad) a.grad[i] = gsum;
    if (a.adam) {
        const float mm = a.beta1 * a.m1[i] + (1.0f - a.beta1) * gsum;
        const float vv = a.beta2 * a.m2[i] + (1.0f - a.beta2) * gsum * gsum;
        a.m1[i] = mm;
        a.m2[i] = vv;
        a.theta[i] -= a.lr * (mm / a.bc1) / (sqrtf(vv / a.bc2) + a.eps);
    }
}

// ---------------------------------------------------------------------------
// training inputs of selected rays
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_gather(const int64_t* __restrict__ ray_id, int64_t n,
                                                    const float* __restrict__ labels, const CamParams* __restrict__ cam,
                                                    int P, int V, int H, int W, float* __restrict__ od,
                                                    int32_t* __restrict__ pose, float* __restrict__ target,
                                                    uint32_t* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t total = (int64_t)P * V * HW;
    const int64_t id = ray_id[i];
    if (id < 0 || id >= total) {
        atomicOr(bad, 1u);
        for (int k = 0; k < 6; ++k) od[i * 6 + k] = 0.0f;
        pose[i] = 0;
        target[i * 2] = 1.0f;
        target[i * 2 + 1] = 0.0f;
        return;
    }
    const int64_t pv = id / HW, pix = id % HW;
    const int p = (int)(pv / V), v = (int)(pv % V);
    float o[3], d[3];
    ray_f32(cam[v], (int)(pix % W), (int)(pix / W), o, d);
    for (int k = 0; k < 3; ++k) {
        od[i * 6 + k] = o[k];
        od[i * 6 + 3 + k] = d[k];
    }
    pose[i] = p;
    target[i * 2] = labels[id * 2];
    target[i * 2 + 1] = labels[id * 2 + 1];
}

// ---------------------------------------------------------------------------
// inference for the rays of the compacted non-empty tiles of a render launch
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_infer_tiles(InferLaunch a) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    WRegs W;
    {
        const bf16x8* P = reinterpret_cast<const bf16x8*>(a.packed);
#pragma unroll
        for (int b = 0; b < kB_W4T; ++b) W.b[b] = P[b * 64 + lane];
    }
    InferBias B;
    load_infer_bias(a.theta, a.m, g, B);
    const uint32_t n_items = *a.n_items;
    const uint32_t nw = gridDim.x * (blockDim.x / 64);
    for (uint32_t idx = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); idx < n_items; idx += nw) {
        const uint32_t item = a.items[idx];
        const int pvi = (int)(item / (uint32_t)a.TPV);
        const int tile = (int)(item % (uint32_t)a.TPV);
        const int pb = pvi / a.V, v = pvi % a.V;
        const int tx = tile % a.TX, ty = tile / a.TX;
        f32x4 c1[4];
        load_pose_bias(a.cbias + (size_t)(a.pose0 + pb) * kHid, g, c1);
        // the ray of the tile pixel `lane` (row-major 8x8); group q reads the
        // inputs of pixels 16 q .. 16 q + 15 from those lanes
        float xl[6];
        ray_f32(a.cam[v], tx * 8 + (lane & 7), ty * 8 + (lane >> 3), xl, xl + 3);
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
            float x[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) x[i] = __shfl(xl[i], 16 * q + r, kWave);
            const float2 y = infer_group(W, B, c1, x, g);
            if (g == 0) reinterpret_cast<float2*>(a.out)[(size_t)idx * 64 + 16 * q + r] = y;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_pose_code(const double* pose, int J, int P, float* code, hipStream_t st) {
    const int n = P * J;
    hipLaunchKernelGGL(k_pose_code, dim3((n + 127) / 128), dim3(128), 0, st, pose, J, P, code);
    return hipGetLastError();
}

hipError_t launch_mlp_prep(const float* theta, const MlpDims& m, const float* code, int P, uint16_t* packed,
                           float* cbias, hipStream_t st) {
    const int n = kPacked + P * kHid;
    hipLaunchKernelGGL(k_mlp_prep, dim3((n + 255) / 256), dim3(256), 0, st, theta, m, code, P, packed, cbias);
    return hipGetLastError();
}

int64_t mlp_pad(int64_t n) { return (n + kChunk - 1) / kChunk * kChunk; }
size_t mlp_scratch_bytes(int64_t n) { return (size_t)kRows * (size_t)mlp_pad(n) * 4; }
int mlp_packed_elems() { return kPacked; }

static unsigned fb_grid(int64_t n_pad) {
    const int64_t groups = n_pad / 16;
    int64_t g = (groups + 3) / 4;
    if (g > 2048) g = 2048;
    return (unsigned)std::max<int64_t>(g, 1);
}
unsigned mlp_loss_parts(int64_t n) { return fb_grid(mlp_pad(n)); }

hipError_t launch_mlp_forward(const uint16_t* packed, const float* theta, const float* cbias, const MlpDims& m,
                              const float* od, const int32_t* pose, int P, int64_t n, float* out, uint32_t* bad,
                              hipStream_t st) {
    FbArgs a{};
    a.P = P;
    a.bad = bad;
    a.packed = packed;
    a.theta = theta;
    a.cbias = cbias;
    a.m = m;
    a.od = od;
    a.pose = pose;
    a.out = out;
    a.n = n;
    a.n_pad = (n + 15) / 16 * 16;
    a.mode = 0;
    hipLaunchKernelGGL(k_mlp_fb, dim3(fb_grid(a.n_pad)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const uint16_t* packed, const float* theta, const float* cbias, const float* code,
                           const MlpDims& m, const float* od, const int32_t* pose, const float* target, int P,
                           int64_t n, float* S, float* part, float* loss_part, uint32_t* bad, const MlpLoss& loss,
                           hipStream_t st) {
    FbArgs a{};
    a.loss = loss;
    a.P = P;
    a.bad = bad;
    a.packed = packed;
    a.theta = theta;
    a.cbias = cbias;
    a.m = m;
    a.od = od;
    a.pose = pose;
    a.target = target;
    a.n = n;
    a.n_pad = mlp_pad(n);
    a.S = S;
    a.loss_part = loss_part;
    a.inv2n = 1.0f / (2.0f * (float)n);
    a.mode = 1;
    hipLaunchKernelGGL(k_mlp_fb, dim3(fb_grid(a.n_pad)), dim3(256), 0, st, a);
    WgArgs w{};
    w.S = S;
    w.n = n;
    w.n_pad = a.n_pad;
    w.od = od;
    w.pose = pose;
    w.code = code;
    w.P = P;
    w.m = m;
    w.part = part;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)(a.n_pad / kChunk)), dim3(256), 0, st, w);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float* part, int64_t n, const MlpDims& m, float* grad, float* theta, float* m1,
                             float* m2, const AdamStep* adam, const float* loss_part, float* loss_out,
                             hipStream_t st) {
    RedArgs a{};
    a.part = part;
    a.nchunks = (int)(mlp_pad(n) / kChunk);
    a.np = m.np;
    a.grad = grad;
    a.theta = theta;
    a.m1 = m1;
    a.m2 = m2;
    a.adam = adam != nullptr;
    if (adam) {
        a.lr = adam->lr;
        a.beta1 = adam->beta1;
        a.beta2 = adam->beta2;
        a.eps = adam->eps;
        a.bc1 = adam->bc1;
        a.bc2 = adam->bc2;
    }
    a.loss_part = loss_part;
    a.nloss = (int)mlp_loss_parts(n);
    a.inv2n = 1.0f / (2.0f * (float)n);
    a.loss_out = loss_out;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((m.np + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mlp_gather(const int64_t* ray_id, int64_t n, const float* labels, const CamParams* cam, int P,
                             int V, int H, int W, float* od, int32_t* pose, float* target, uint32_t* bad,
                             hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ray_id, n, labels, cam, P,
                       V, H, W, od, pose, target, bad);
    return hipGetLastError();
}

hipError_t launch_mlp_infer_tiles(const InferLaunch& a, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_infer_tiles, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace art
