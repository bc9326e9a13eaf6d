// The pixels whose 8x8 tile has no brick list (no voxel on their ray): F = 0,
// A = 0, T = 1, depth +inf, the empty interval label (1, 0) and no hits.
// Written in groups of 4 consecutive pixels of a row (images whose width is
// a multiple of 4, 16-byte aligned maps) by the vectorised background kernel,
// or - for the forward maps - by the compositing kernel's own waves between
// their tiles, so that the stores overlap its compositing.
#pragma once

#include "device_util.h"

namespace art {

struct BgArgs {
    int V, Vg, ngroups, H, W, C, TX, TPV;
    int debug_view;   // -1: all views
    const uint32_t* ovf;
    const uint32_t* tile_start;
    const uint32_t* tile_end;
    float* out_feat;
    float* out_alpha;
    float* out_tfinal;
    float* labels;
    float* out_depth;
    int32_t* hit_count;
};

// 4-pixel group q (< H * W / 4, row-major) of map pvi (pose * V + view) of
// the launch.  Returns the pixels written (0 or 4).
__device__ inline int bg_group4(const BgArgs& g, uint32_t pvi, uint32_t q) {
    const size_t HW = (size_t)g.H * g.W;
    const uint32_t pix = q * 4u;
    const int py = (int)(pix / (uint32_t)g.W), px = (int)(pix % (uint32_t)g.W);
    const int pb = (int)pvi / g.V, v = (int)pvi % g.V;
    if (g.debug_view >= 0 && v != g.debug_view) return 0;
    if (g.ovf[2 * ((size_t)pb * g.ngroups + v / g.Vg)]) return 0;   // re-run later by the host
    const size_t item = (size_t)pvi * g.TPV + (size_t)(py >> 3) * g.TX + (px >> 3);
    if (g.tile_end[item] > g.tile_start[item]) return 0;             // rendered by k_render
    const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (g.out_feat)
        for (int c = 0; c < g.C; ++c) store_stream4(g.out_feat + ((size_t)pvi * g.C + c) * HW + pix, zero);
    if (g.out_alpha) store_stream4(g.out_alpha + (size_t)pvi * HW + pix, zero);
    if (g.out_tfinal) store_stream4(g.out_tfinal + (size_t)pvi * HW + pix, make_float4(1.0f, 1.0f, 1.0f, 1.0f));
    if (g.labels) {
        float4* l = reinterpret_cast<float4*>(g.labels + ((size_t)pvi * HW + pix) * 2);
        l[0] = make_float4(1.0f, 0.0f, 1.0f, 0.0f);
        l[1] = make_float4(1.0f, 0.0f, 1.0f, 0.0f);
    }
    if (g.out_depth)
        reinterpret_cast<float4*>(g.out_depth + (size_t)pvi * HW)[q] = make_float4(INFINITY, INFINITY, INFINITY, INFINITY);
    if (g.hit_count) reinterpret_cast<int4*>(g.hit_count + (size_t)0)[q] = make_int4(0, 0, 0, 0);
    return 4;
}

// 4-pixel groups of one background chunk taken by a single wave.
constexpr uint32_t kBgChunkGroups = 256;

}  // namespace art
