// Tile work distribution of the compositing pass.
//
//   k_tile_compact : one thread per tile slot (Morton order within each view);
//                    tiles whose brick list is not empty are appended to the work
//                    list in slot order within each workgroup's range of slots
//                    (wave ballots, counts in LDS, one atomic per workgroup
//                    range), so the persistent compositing waves only ever take
//                    tiles with work.
//   k_background   : one thread per pixel; the pixels of an empty tile get
//                    F = 0, A = 0, T = 1 (no voxel on their ray), and the
//                    empty interval label (1, 0) in a label pass.
#include "background.h"
#include "device_util.h"
#include "internal.h"

namespace art {

struct TileGeom {
    int Pb, V, Vg, ngroups, TX, TY, TPV, H, W, C;
    uint32_t tiles_pow4;
    int debug_view;   // -1: all views
};

__device__ inline bool tile_slot(const TileGeom& g, const uint32_t* ovf, uint64_t i, uint32_t* item,
                                 int* tx, int* ty, int* pvi) {
    const uint64_t total = (uint64_t)g.Pb * g.V * g.tiles_pow4;
    if (i >= total) return false;
    *pvi = (int)(i / g.tiles_pow4);
    const uint32_t mt = (uint32_t)(i % g.tiles_pow4);
    *tx = (int)compact2(mt);
    *ty = (int)compact2(mt >> 1);
    if (*tx >= g.TX || *ty >= g.TY) return false;
    const int pb = *pvi / g.V;
    const int v = *pvi % g.V;
    if (g.debug_view >= 0 && v != g.debug_view) return false;
    if (ovf[2 * ((size_t)pb * g.ngroups + v / g.Vg)]) return false;   // re-run later by the host
    *item = (uint32_t)((uint64_t)*pvi * g.TPV + (uint64_t)*ty * g.TX + *tx);
    return true;
}

// A workgroup compacts kCompactIters x 256 consecutive tile slots: the waves
// count their slots with work (one ballot per iteration), the workgroup takes
// its range of the work list with one atomic, and every item is written at
// its slot-order position within the range.
constexpr int kCompactThreads = 256;
constexpr int kCompactWaves = kCompactThreads / kWave;
constexpr int kCompactIters = 16;
__global__ __launch_bounds__(kCompactThreads) void k_tile_compact(TileGeom g, const uint32_t* __restrict__ ovf,
                                                                  const uint32_t* __restrict__ tstart,
                                                                  const uint32_t* __restrict__ tend,
                                                                  uint32_t* __restrict__ items,
                                                                  uint32_t* __restrict__ n_items) {
    __shared__ uint32_t s_cnt[kCompactIters][kCompactWaves];
    __shared__ uint32_t s_base;
    const uint64_t total = (uint64_t)g.Pb * g.V * g.tiles_pow4;
    const uint64_t span = (uint64_t)kCompactIters * kCompactThreads;
    const int w = (int)threadIdx.x / kWave;
    const int lane = lane_id();
    for (uint64_t b0 = (uint64_t)blockIdx.x * span; b0 < total; b0 += (uint64_t)gridDim.x * span) {
        uint64_t mask[kCompactIters];
        uint32_t item[kCompactIters];
#pragma unroll
        for (int k = 0; k < kCompactIters; ++k) {
            const uint64_t i = b0 + (uint64_t)k * kCompactThreads + threadIdx.x;
            int tx, ty, pvi;
            item[k] = 0;
            bool work = tile_slot(g, ovf, i, &item[k], &tx, &ty, &pvi);
            work = work && tend[item[k]] > tstart[item[k]];
            mask[k] = __ballot(work);
            if (lane == 0) s_cnt[k][w] = (uint32_t)__popcll(mask[k]);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int k = 0; k < kCompactIters; ++k)
                for (int q = 0; q < kCompactWaves; ++q) tot += s_cnt[k][q];
            s_base = tot ? atomicAdd(n_items, tot) : 0u;
        }
        __syncthreads();
        // slot order: iteration k, then wave q, then lane
        uint32_t off = s_base;
#pragma unroll
        for (int k = 0; k < kCompactIters; ++k) {
            for (int q = 0; q < w; ++q) off += s_cnt[k][q];
            if ((mask[k] >> lane) & 1ull) items[off + (uint32_t)__popcll(mask[k] & lanemask_lt())] = item[k];
            for (int q = w; q < kCompactWaves; ++q) off += s_cnt[k][q];
        }
        __syncthreads();   // s_cnt and s_base are rewritten by the next range
    }
}

// One thread per pixel of every (pose, view) map, row-major so each output
// plane is written in full 256-byte runs; pixels of tiles with a brick list are
// left to the compositing kernel.
__global__ __launch_bounds__(256) void k_background(TileGeom g, const uint32_t* __restrict__ ovf,
                                                    const uint32_t* __restrict__ tstart,
                                                    const uint32_t* __restrict__ tend,
                                                    float* __restrict__ out_feat, float* __restrict__ out_alpha,
                                                    float* __restrict__ out_tfinal, float* __restrict__ labels,
                                                    float* __restrict__ out_depth, int32_t* __restrict__ hit_count,
                                                    unsigned long long* __restrict__ stats) {
    const size_t HW = (size_t)g.H * g.W;
    const uint64_t total = (uint64_t)g.Pb * g.V * HW;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long nrays = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint32_t pvi = (uint32_t)(i / HW);
        const size_t pix = (size_t)(i % HW);
        const int py = (int)(pix / g.W), px = (int)(pix % g.W);
        const int pb = (int)pvi / g.V, v = (int)pvi % g.V;
        if (g.debug_view >= 0 && v != g.debug_view) continue;
        if (ovf[2 * ((size_t)pb * g.ngroups + v / g.Vg)]) continue;   // re-run later by the host
        const size_t item = (size_t)pvi * g.TPV + (size_t)(py >> 3) * g.TX + (px >> 3);
        if (tend[item] > tstart[item]) continue;                      // rendered by k_render
        ++nrays;
        if (out_feat)
            for (int c = 0; c < g.C; ++c) store_stream(&out_feat[((size_t)pvi * g.C + c) * HW + pix], 0.0f);
        if (out_alpha) store_stream(&out_alpha[(size_t)pvi * HW + pix], 0.0f);
        if (out_tfinal) store_stream(&out_tfinal[(size_t)pvi * HW + pix], 1.0f);
        if (labels) reinterpret_cast<float2*>(labels)[(size_t)pvi * HW + pix] = make_float2(1.0f, 0.0f);
        if (out_depth) out_depth[(size_t)pvi * HW + pix] = INFINITY;
        if (hit_count) hit_count[pix] = 0;
    }
    if (stats) {   // one atomic per workgroup
        __shared__ unsigned long long part[256 / kWave];
        const unsigned long long w = wave_sum(nrays);
        if (lane_id() == 0) part[threadIdx.x / kWave] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long t = part[0] + part[1] + part[2] + part[3];
            if (t) atomicAdd(&stats[0], t);
        }
    }
}

// Same as k_background for images whose width is a multiple of 4: a thread
// owns 4 consecutive pixels of a row (one tile) and writes 16-byte vectors.
__global__ __launch_bounds__(256) void k_background4(BgArgs g, uint64_t total, unsigned long long* __restrict__ stats) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long nrays = 0;
    const uint64_t HW4 = (uint64_t)g.H * g.W / 4;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
        nrays += (unsigned long long)bg_group4(g, (uint32_t)(i / HW4), (uint32_t)(i % HW4));
    if (stats) {   // one atomic per workgroup
        __shared__ unsigned long long part[256 / kWave];
        const unsigned long long w = wave_sum(nrays);
        if (lane_id() == 0) part[threadIdx.x / kWave] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long t = part[0] + part[1] + part[2] + part[3];
            if (t) atomicAdd(&stats[0], t);
        }
    }
}

// Workgroups of the vectorised background kernel (at most): enough for one
// 4-pixel group per thread at 30 poses x 8 views of 512^2 (a smaller grid
// that loops measured 2 % slower on this stage).
#ifndef ART_BG_BLOCKS
#define ART_BG_BLOCKS 65536
#endif

BgArgs bg_args(const TileLaunch& t, const TileGeom& g) {
    BgArgs b;
    b.V = g.V;
    b.Vg = g.Vg;
    b.ngroups = g.ngroups;
    b.H = g.H;
    b.W = g.W;
    b.C = g.C;
    b.TX = g.TX;
    b.TPV = g.TPV;
    b.debug_view = g.debug_view;
    b.ovf = t.ovf;
    b.tile_start = t.tile_start;
    b.tile_end = t.tile_end;
    b.out_feat = t.out_feat;
    b.out_alpha = t.out_alpha;
    b.out_tfinal = t.out_tfinal;
    b.labels = t.labels;
    b.out_depth = t.out_depth;
    b.hit_count = t.hit_count;
    return b;
}

bool background_vectorised(const TileLaunch& t) {
    return (t.W % 4) == 0 &&
           ((reinterpret_cast<uintptr_t>(t.out_feat) | reinterpret_cast<uintptr_t>(t.out_alpha) |
             reinterpret_cast<uintptr_t>(t.out_tfinal) | reinterpret_cast<uintptr_t>(t.labels) |
             reinterpret_cast<uintptr_t>(t.out_depth) | reinterpret_cast<uintptr_t>(t.hit_count)) &
            15u) == 0;
}

hipError_t launch_tiles(const TileLaunch& t, hipStream_t st) {
    TileGeom g;
    g.Pb = t.Pb;
    g.V = t.V;
    g.Vg = t.Vg;
    g.ngroups = t.ngroups;
    g.TX = (t.W + 7) / 8;
    g.TY = (t.H + 7) / 8;
    g.TPV = g.TX * g.TY;
    g.H = t.H;
    g.W = t.W;
    g.C = t.C;
    g.tiles_pow4 = t.tiles_pow4;
    g.debug_view = t.debug_view;
    const uint64_t total = (uint64_t)g.Pb * g.V * g.tiles_pow4;
    hipError_t e = launch_fill_u32(t.counters, 0u, 16, st);   // n_items, queue heads
    if (e != hipSuccess) return e;
    const uint64_t span = (uint64_t)kCompactIters * kCompactThreads;
    uint64_t blocks = (total + span - 1) / span;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_tile_compact, dim3((unsigned)blocks), dim3(kCompactThreads), 0, st, g, t.ovf, t.tile_start,
                       t.tile_end, t.items, t.counters);
    if (t.out_feat || t.hit_count || t.labels) {
        const uint64_t pixels = (uint64_t)g.Pb * g.V * g.H * g.W;
        uint64_t wblocks = (pixels + 255) / 256;
        if (wblocks > 16384) wblocks = 16384;
        if (wblocks < 1) wblocks = 1;
        // 16-byte stores when rows hold whole 4-pixel groups (and the caller's maps are
        // 16-byte aligned, as device allocations are)
        const bool vec = background_vectorised(t);
        if (vec) {
            if (!t.bg_in_render) {
                uint64_t vblocks = (pixels / 4 + 255) / 256;
                if (vblocks > ART_BG_BLOCKS) vblocks = ART_BG_BLOCKS;
                if (vblocks < 1) vblocks = 1;
                hipLaunchKernelGGL(k_background4, dim3((unsigned)vblocks), dim3(256), 0, st, bg_args(t, g), pixels / 4,
                                   t.stats);
            }
        } else {
            hipLaunchKernelGGL(k_background, dim3((unsigned)wblocks), dim3(256), 0, st, g, t.ovf, t.tile_start,
                               t.tile_end, t.out_feat, t.out_alpha, t.out_tfinal, t.labels, t.out_depth, t.hit_count, t.stats);
        }
    }
    return hipGetLastError();
}

}  // namespace art
