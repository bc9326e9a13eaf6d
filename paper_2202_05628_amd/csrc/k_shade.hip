// Neural shading network G, the "Light" variant of Section 3.1 / Section 6
// ("Neural Shading", runtime analysis): one encoder-decoder (U-Net) branch that
// turns the feature map F into an RGB image and an opacity map (the opacity
// branch removed, one output channel added), in half precision.
//
// Layout: activations NHWC in FP16 (channels innermost, multiples of 32);
// weights [3][3][Cout][Cin] FP16; bias FP32.  Every 3x3 convolution (pad 1,
// stride 1, bias, optional ReLU) is an implicit GEMM on the matrix cores:
// D[cout][pixel] += W[cout][k] X[k][pixel] over k = (ky, kx, cin), with
// v_mfma_f32_16x16x32_f16 (FP16 operands, FP32 accumulation).  A workgroup
// (4 waves) computes TP consecutive pixels of one image row for TC output
// channels (the tile is chosen per layer, see ConvTile); per 32-channel chunk
// and kernel row (a stage) it stages the input row (with its halo) and the
// 3 x TC weight rows in LDS, the global loads of the next stage in flight
// while the matrix cores work on the current one.  The decoder's input
// (skip connection, nearest-upsampled deeper level) is read by the staging
// directly: channels [0, C1) from the same-resolution source, [C1, C1 + C2)
// from the half-resolution one at (y/2, x/2), so neither the upsampled tensor
// nor the concatenation is materialised.
//
// MFMA operand layout of the 16x16x32 shape (wave64): lane l holds
//   A[l % 16][8 (l / 16) + e], B[8 (l / 16) + e][l % 16] for e = 0..7 and
//   D[4 (l / 16) + e][l % 16] for e = 0..3.
#include "device_util.h"
#include "internal.h"
#include "shade.h"

namespace art {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float fl4 __attribute__((ext_vector_type(4)));

constexpr int kPix = 40;            // halves per staged pixel / weight row: 32 channels + 8 (bank spread)
constexpr int kConvWaves = 4;
#ifndef ART_CONV_XCD
#define ART_CONV_XCD 1
#endif
constexpr uint32_t kXcds = 8;
// Fourth descriptor word of a raw buffer resource (32-bit data format, no
// swizzle) for CDNA3 / CDNA4.
constexpr int kBufferFlags = 0x00020000;

// Workgroup tile: 4 waves, WC of them side by side over output channels and
// 4 / WC over pixels; each wave computes PB blocks of 16 pixels x NCB blocks
// of 16 output channels, so a workgroup covers TP = 16 PB (4 / WC) pixels of
// a row and TC = 16 NCB WC output channels.  A larger wave tile reads fewer
// LDS operands per matrix product (PB + NCB reads for PB NCB products).
template <int NCB, int PB, int WC>
struct ConvTile {
    static constexpr int WP = kConvWaves / WC;
    static constexpr int TP = 16 * PB * WP;
    static constexpr int TC = 16 * NCB * WC;
    static constexpr int lds_bytes = ((TP + 2) + 3 * TC) * kPix * 2;
    static constexpr int in_it = ((TP + 2) * 4 + 255) / 256;   // staged 16-byte vectors per thread
    static constexpr int w_it = (3 * TC * 4 + 255) / 256;
    // registers per lane: accumulators, B operands, staged loads, their offsets, the rest
    static constexpr int vgprs = 4 * PB * NCB + 4 * PB + 4 * (in_it + w_it) + 2 * in_it + w_it + 24;
    static constexpr int by_lds = 163840 / lds_bytes;   // resident workgroups per CU (160 KB LDS)
    static constexpr int by_regs = 512 / vgprs;
    static constexpr int waves_per_simd = by_lds < by_regs ? (by_lds < 4 ? by_lds : 4) : (by_regs < 4 ? by_regs : 4);
    static_assert(waves_per_simd >= 1, "convolution tile does not fit one CU");
};

template <int NCB, int PB, int WC, bool HEAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ConvTile<NCB, PB, WC>::waves_per_simd)))
void k_conv3x3(ConvLaunch a, ConvHead hd) {
    using Tl = ConvTile<NCB, PB, WC>;
    constexpr int kConvPB = PB;
    constexpr int kConvTP = Tl::TP;
    const _Float16* src1 = reinterpret_cast<const _Float16*>(a.src1);
    const _Float16* src2 = reinterpret_cast<const _Float16*>(a.src2);
    const _Float16* wgt = reinterpret_cast<const _Float16*>(a.wgt);
    _Float16* outp = reinterpret_cast<_Float16*>(a.out);
    constexpr int TC = Tl::TC;                           // output channels per workgroup
    constexpr int kInVec = (kConvTP + 2) * 4;            // 16-byte vectors of a staged input row
    constexpr int kWVec = 3 * TC * 4;                    // 16-byte vectors of a staged kernel row
    constexpr int kInIt = (kInVec + 255) / 256;
    constexpr int kWIt = (kWVec + 255) / 256;
    __shared__ __align__(16) _Float16 s_in[(kConvTP + 2) * kPix];
    __shared__ __align__(16) _Float16 s_w[3 * TC * kPix];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int wp = wave % Tl::WP, wc = wave / Tl::WP;   // pixel / channel position of the wave
    const int lane = tid & 63;
    // Workgroups are dealt to the 8 XCDs in turn (XCD = linear id mod 8);
    // renumbering them so that each XCD gets a contiguous range of (pixel
    // tile, row, image) keeps the neighbouring rows that read the same input
    // rows, and the weights, in one XCD's L2.
    int bx = blockIdx.x, y = blockIdx.y, bz = blockIdx.z;
#if ART_CONV_XCD
    {
        const uint32_t gx = gridDim.x, gy = gridDim.y;
        const uint32_t nb = gx * gy * gridDim.z;
        const uint32_t hw = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
        const uint32_t q = nb / kXcds, r = nb % kXcds, k = hw % kXcds;
        const uint32_t L = k * q + (k < r ? k : r) + hw / kXcds;
        bx = (int)(L % gx);
        y = (int)((L / gx) % gy);
        bz = (int)(L / (gx * gy));
    }
#endif
    const int x0 = bx * kConvTP;
    const int ntc = a.Cout / TC;
    const int ct = bz % ntc;
    const int n = bz / ntc;
    const int Cin = a.C1 + a.C2;
    const int H2 = a.H >> 1, W2 = a.W >> 1;
    const int nstage = (Cin / 32) * 3;                   // (32-channel chunk, kernel row) stages
    fl4 acc[kConvPB][NCB];
#pragma unroll
    for (int p = 0; p < kConvPB; ++p)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[p][c] = fl4{0.0f, 0.0f, 0.0f, 0.0f};

    // The image's input tensors and the weights are read through buffer
    // resources: a load at an offset beyond a resource returns zeros, which is
    // the zero padding of the halo pixels and of the rows above and below the
    // image.  Offsets are bytes: a lane part (fixed over the stages) plus a
    // wave-uniform stage part, each either inside the resource (< 2^30 bytes,
    // checked by the launcher) or kOOB, so their sum cannot wrap.
    constexpr uint32_t kOOB = 1u << 30;
    const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(src1 + (size_t)n * a.H * a.W * a.C1), (short)0, a.H * a.W * a.C1 * 2, kBufferFlags);
    const __amdgpu_buffer_rsrc_t rs2 =
        a.C2 ? __builtin_amdgcn_make_buffer_rsrc((void*)(src2 + (size_t)n * H2 * W2 * a.C2), (short)0,
                                                 H2 * W2 * a.C2 * 2, kBufferFlags)
             : rs1;
    const __amdgpu_buffer_rsrc_t rsw =
        __builtin_amdgcn_make_buffer_rsrc((void*)wgt, (short)0, 9 * a.Cout * Cin * 2, kBufferFlags);
    // input vector v = tid + 256 j is channel quarter v % 4 of pixel v / 4 of
    // the staged row (x = x0 - 1 + v / 4); weight vector v is quarter v % 4 of
    // kernel-row entry v / 4 = (kx, output channel)
    uint32_t in_b1[kInIt], in_b2[kInIt];
#pragma unroll
    for (int j = 0; j < kInIt; ++j) {
        const int v = tid + 256 * j;
        const int q = v & 3;
        const int xx = x0 - 1 + (v >> 2);
        const bool ok = v < kInVec && xx >= 0 && xx < a.W;
        in_b1[j] = ok ? (uint32_t)(xx * a.C1 + 8 * q) * 2u : kOOB;
        in_b2[j] = ok ? (uint32_t)((xx >> 1) * a.C2 + 8 * q) * 2u : kOOB;
    }
    uint32_t w_b[kWIt];
#pragma unroll
    for (int j = 0; j < kWIt; ++j) {
        const int v = tid + 256 * j;
        const int q = v & 3, r = v >> 2;
        const int co = r % TC, kx = r / TC;
        w_b[j] = v < kWVec ? (uint32_t)((kx * a.Cout + ct * TC + co) * Cin + 8 * q) * 2u : kOOB;
    }

    // Software pipeline: the global loads of stage s + 1 go to registers while
    // the matrix cores work on stage s from LDS.
    half8 rin[kInIt], rw[kWIt];
    auto load_stage = [&](int st) {
        const int c0 = (st / 3) * 32, ky = st % 3;
        const int yy = y + ky - 1;
        const bool up = c0 >= a.C1;
        const uint32_t row = (yy < 0 || yy >= a.H) ? kOOB
                             : up ? (uint32_t)(((yy >> 1) * W2) * a.C2 + (c0 - a.C1)) * 2u
                                  : (uint32_t)((yy * a.W) * a.C1 + c0) * 2u;
#pragma unroll
        for (int j = 0; j < kInIt; ++j)
            rin[j] = __builtin_bit_cast(half8, __builtin_amdgcn_raw_buffer_load_b128(up ? rs2 : rs1,
                                                                                     (up ? in_b2[j] : in_b1[j]) + row, 0, 0));
        const uint32_t wrow = (uint32_t)(ky * 3 * a.Cout * Cin + c0) * 2u;
#pragma unroll
        for (int j = 0; j < kWIt; ++j)
            rw[j] = __builtin_bit_cast(half8, __builtin_amdgcn_raw_buffer_load_b128(rsw, w_b[j] + wrow, 0, 0));
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int j = 0; j < kInIt; ++j) {
            const int v = tid + 256 * j;
            if (v < kInVec) *reinterpret_cast<half8*>(s_in + (v >> 2) * kPix + 8 * (v & 3)) = rin[j];
        }
#pragma unroll
        for (int j = 0; j < kWIt; ++j) {
            const int v = tid + 256 * j;
            if (v < kWVec) *reinterpret_cast<half8*>(s_w + (v >> 2) * kPix + 8 * (v & 3)) = rw[j];
        }
    };

    load_stage(0);
    store_stage();
    __syncthreads();
    for (int st = 0; st < nstage; ++st) {
        if (st + 1 < nstage) load_stage(st + 1);
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            half8 bx[kConvPB];
#pragma unroll
            for (int p = 0; p < kConvPB; ++p) {
                const int px = (wp * kConvPB + p) * 16 + (lane & 15) + kx;
                bx[p] = *reinterpret_cast<const half8*>(s_in + px * kPix + 8 * (lane >> 4));
            }
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                const half8 aw =
                    *reinterpret_cast<const half8*>(s_w + (kx * TC + (wc * NCB + c) * 16 + (lane & 15)) * kPix +
                                                    8 * (lane >> 4));
#pragma unroll
                for (int p = 0; p < kConvPB; ++p)
                    acc[p][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aw, bx[p], acc[p][c], 0, 0, 0);
            }
        }
        __syncthreads();   // every wave has read this stage
        if (st + 1 < nstage) {
            store_stage();
            __syncthreads();
        }
    }
    if constexpr (HEAD) {
        // The network's last convolution (32 output channels, one channel
        // tile) with the 1x1 head fused: its outputs after bias and ReLU,
        // rounded to FP16 as a stored activation is, enter
        // out_k = sigmoid(b_k + sum_c w_kc x_c) in FP32 directly.  Lane group
        // g = lane / 16 holds channels 16 c + 4 g + e of its pixel; the four
        // groups' partial sums are added across lanes, and group g writes
        // output k = g.
        const int g = lane >> 4;
        const size_t HW = (size_t)a.H * a.W;
        // this lane's channels 16 c + 4 g + e: their biases and head weights,
        // loaded once (the output stores could alias them)
        fl4 bv[NCB], wv[NCB][4];
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            bv[c] = *reinterpret_cast<const fl4*>(a.bias + c * 16 + 4 * g);
#pragma unroll
            for (int k = 0; k < 4; ++k) wv[c][k] = *reinterpret_cast<const fl4*>(hd.w + k * 32 + c * 16 + 4 * g);
        }
        const float bg = hd.b[g];
#pragma unroll
        for (int p = 0; p < kConvPB; ++p) {
            const int x = x0 + (wp * kConvPB + p) * 16 + (lane & 15);
            float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[p][c][e] + bv[c][e];
                    if (a.relu) v = fmaxf(v, 0.0f);
                    v = (float)(_Float16)v;
#pragma unroll
                    for (int k = 0; k < 4; ++k) part[k] = fmaf(wv[c][k][e], v, part[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                part[k] += __shfl_xor(part[k], 16, kWave);
                part[k] += __shfl_xor(part[k], 32, kWave);
            }
            const float z = bg + (g == 0 ? part[0] : g == 1 ? part[1] : g == 2 ? part[2] : part[3]);
            if (x < a.W) hd.out[((size_t)n * 4 + g) * HW + (size_t)y * a.W + x] = 1.0f / (1.0f + expf(-z));
        }
        return;
    }
    // epilogue: bias, ReLU, FP16 NHWC store (4 consecutive channels per lane)
#pragma unroll
    for (int p = 0; p < kConvPB; ++p) {
        const int x = x0 + (wp * kConvPB + p) * 16 + (lane & 15);
        if (x >= a.W) continue;
        _Float16* o = outp + (((size_t)n * a.H + y) * a.W + x) * a.Cout + ct * TC;
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            const int co = (wc * NCB + c) * 16 + 4 * (lane >> 4);
            half4 h;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = acc[p][c][e] + a.bias[ct * TC + co + e];
                if (a.relu) v = fmaxf(v, 0.0f);
                h[e] = (_Float16)v;
            }
            *reinterpret_cast<half4*>(o + co) = h;
        }
    }
}

template <int NCB, int PB, int WC, bool HEAD = false>
static void conv_launch(const ConvLaunch& a, hipStream_t st, const ConvHead& hd = ConvHead{}) {
    using Tl = ConvTile<NCB, PB, WC>;
    const dim3 grid((unsigned)((a.W + Tl::TP - 1) / Tl::TP), (unsigned)a.H, (unsigned)(a.N * (a.Cout / Tl::TC)));
    hipLaunchKernelGGL((k_conv3x3<NCB, PB, WC, HEAD>), grid, dim3(256), 0, st, a, hd);
}

template <int NCB, int WC>
static void conv_launch_pb(const ConvLaunch& a, int pb, hipStream_t st) {
    switch (pb) {
        case 1: conv_launch<NCB, 1, WC>(a, st); break;
        case 2: conv_launch<NCB, 2, WC>(a, st); break;
        default: conv_launch<NCB, 4, WC>(a, st); break;
    }
}

// Tile choice: 64 output channels per wave when Cout allows (else 32), the
// waves spread over as many channel tiles as Cout holds (up to 4), then the
// widest pixel tile (up to 4 blocks of 16 per wave) that the row fills.  (8
// blocks per wave for the 32-channel layers ran 10-20 % longer: two waves per
// SIMD.)
static bool conv_args_ok(const ConvLaunch& a) {
    if ((a.C1 % 32) || (a.C2 % 32) || a.C1 <= 0 || (a.C2 > 0 && !a.src2)) return false;
    // buffer resources: one image of each input, and the weights, below 2^30 bytes
    const int64_t lim = (int64_t)1 << 30;
    if ((int64_t)a.H * a.W * a.C1 * 2 >= lim || (int64_t)(a.H / 2) * (a.W / 2) * a.C2 * 2 >= lim ||
        (int64_t)9 * a.Cout * (a.C1 + a.C2) * 2 >= lim)
        return false;
    return a.Cout % 32 == 0;
}

hipError_t launch_conv3x3_head(const ConvLaunch& a, const ConvHead& h, hipStream_t st) {
    if (!conv_args_ok(a) || a.Cout != 32 || !h.w || !h.b || !h.out) return hipErrorInvalidValue;
    if (a.W >= 256) conv_launch<2, 4, 1, true>(a, st, h);
    else if (a.W >= 128) conv_launch<2, 2, 1, true>(a, st, h);
    else conv_launch<2, 1, 1, true>(a, st, h);
    return hipGetLastError();
}

hipError_t launch_conv3x3(const ConvLaunch& a, hipStream_t st) {
    if (!conv_args_ok(a)) return hipErrorInvalidValue;
    if (a.Cout % 64) {   // 32 output channels per workgroup, 4 waves over pixels
        if (a.W >= 256) conv_launch<2, 4, 1>(a, st);
        else if (a.W >= 128) conv_launch<2, 2, 1>(a, st);
        else conv_launch<2, 1, 1>(a, st);
        return hipGetLastError();
    }
    const int tiles = a.Cout / 64;
    const int wc = tiles % 4 == 0 ? 4 : (tiles % 2 == 0 ? 2 : 1);
    const int wp = kConvWaves / wc;
    int pb = 4;
    while (pb > 1 && 16 * pb * wp > a.W) pb >>= 1;
    if (wc == 4) conv_launch_pb<4, 4>(a, pb, st);
    else if (wc == 2) conv_launch_pb<4, 2>(a, pb, st);
    else conv_launch_pb<4, 1>(a, pb, st);
    return hipGetLastError();
}

// Planar FP32 feature maps [N][C][H][W] -> NHWC FP16 with 32 channels (C <= 32,
// zero padded).  A workgroup converts 256 consecutive pixels of one image
// through LDS: each channel plane is read with one coalesced 1 KB row per
// wave, and the 64-byte pixel rows are written as contiguous 4 KB blocks.
constexpr int kNhwcPix = 256;
constexpr int kNhwcPitch = 40;   // halves per staged pixel (32 channels + 8: 16-byte aligned rows)
__global__ __launch_bounds__(256) void k_to_nhwc(const float* __restrict__ F, int C, int HW, int blocks_per_image,
                                                 _Float16* __restrict__ out) {
    __shared__ __align__(16) _Float16 s[kNhwcPix * kNhwcPitch];
    const int n = blockIdx.x / blocks_per_image;
    const int p0 = (blockIdx.x % blocks_per_image) * kNhwcPix;
    const int t = threadIdx.x;
    const int pix = p0 + t;
    const float* f = F + (size_t)n * C * HW;
#pragma unroll 4
    for (int c = 0; c < 32; c += 2) {
        const float a = (pix < HW && c < C) ? f[(size_t)c * HW + pix] : 0.0f;
        const float b = (pix < HW && c + 1 < C) ? f[(size_t)(c + 1) * HW + pix] : 0.0f;
        s[t * kNhwcPitch + c] = (_Float16)a;
        s[t * kNhwcPitch + c + 1] = (_Float16)b;
    }
    __syncthreads();
    _Float16* o = out + ((size_t)n * HW + p0) * 32;
#pragma unroll
    for (int r = 0; r < kNhwcPix * 4 / 256; ++r) {
        const int v = r * 256 + t;               // 16-byte chunk v % 4 of pixel v / 4
        const int px = v >> 2, q = v & 3;
        if (p0 + px < HW)
            *reinterpret_cast<half8*>(o + (size_t)px * 32 + 8 * q) =
                *reinterpret_cast<const half8*>(s + px * kNhwcPitch + 8 * q);
    }
}

// 2x2 max pooling of NHWC FP16 (H, W even), 8 channels per thread.
__global__ __launch_bounds__(256) void k_maxpool2(const _Float16* __restrict__ in, int N, int H, int W, int C,
                                                  _Float16* __restrict__ out) {
    const int H2 = H >> 1, W2 = W >> 1, C8 = C >> 3;
    const size_t total = (size_t)N * H2 * W2 * C8;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(i % C8);
        const size_t r = i / C8;
        const int x = (int)(r % W2), y = (int)((r / W2) % H2);
        const size_t n = r / ((size_t)W2 * H2);
        const _Float16* b = in + ((n * H + 2 * y) * W + 2 * x) * C + 8 * c8;
        half8 m = *reinterpret_cast<const half8*>(b);
        const half8 v1 = *reinterpret_cast<const half8*>(b + C);
        const half8 v2 = *reinterpret_cast<const half8*>(b + (size_t)W * C);
        const half8 v3 = *reinterpret_cast<const half8*>(b + (size_t)W * C + C);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            _Float16 t = m[e] > v1[e] ? m[e] : v1[e];
            t = t > v2[e] ? t : v2[e];
            m[e] = t > v3[e] ? t : v3[e];
        }
        *reinterpret_cast<half8*>(out + i * 8) = m;
    }
}

// Output head: 1x1 convolution of the Cin = 32 channel decoder output to 4
// channels (RGB, opacity) and a sigmoid; planar FP32 [N][4][H][W].
__global__ __launch_bounds__(256) void k_head(const _Float16* __restrict__ in, int N, int H, int W,
                                              const float* __restrict__ w, const float* __restrict__ b,
                                              float* __restrict__ out) {
    __shared__ float sw[4 * 32 + 4];
    for (int i = threadIdx.x; i < 4 * 32 + 4; i += blockDim.x) sw[i] = i < 128 ? w[i] : b[i - 128];
    __syncthreads();
    const size_t HW = (size_t)H * W;
    const size_t total = (size_t)N * HW;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const half8* p = reinterpret_cast<const half8*>(in + i * 32);
        float x[32];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const half8 v = p[q];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[8 * q + e] = (float)v[e];
        }
        const size_t n = i / HW, pix = i % HW;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float s = sw[128 + o];
#pragma unroll
            for (int c = 0; c < 32; ++c) s = fmaf(sw[o * 32 + c], x[c], s);
            out[(n * 4 + o) * HW + pix] = 1.0f / (1.0f + expf(-s));
        }
    }
}

static unsigned grid_for(size_t total) {
    size_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_to_nhwc(const float* F, int N, int C, int H, int W, int Cp, uint16_t* out, hipStream_t st) {
    if (Cp != 32 || C < 1 || C > 32) return hipErrorInvalidValue;
    const int HW = H * W;
    const int bpi = (HW + kNhwcPix - 1) / kNhwcPix;
    hipLaunchKernelGGL(k_to_nhwc, dim3((unsigned)(N * bpi)), dim3(256), 0, st, F, C, HW, bpi,
                       reinterpret_cast<_Float16*>(out));
    return hipGetLastError();
}

hipError_t launch_maxpool2(const uint16_t* in, int N, int H, int W, int C, uint16_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_maxpool2, dim3(grid_for((size_t)N * (H / 2) * (W / 2) * (C / 8))), dim3(256), 0, st,
                       reinterpret_cast<const _Float16*>(in), N, H, W, C, reinterpret_cast<_Float16*>(out));
    return hipGetLastError();
}

hipError_t launch_head(const uint16_t* in, int N, int H, int W, const float* w, const float* b, float* out,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_head, dim3(grid_for((size_t)N * H * W)), dim3(256), 0, st,
                       reinterpret_cast<const _Float16*>(in), N, H, W, w, b, out);
    return hipGetLastError();
}

}  // namespace art
