// Posed-octree rebuild (Section 3.1: the octree is rebuilt for every pose;
// leaves warped onto one cell collide and one of them is kept: the smallest
// canonical leaf index).
//
// The result is a two-level octree: bricks (the level 3 above the leaves) with
// a 512-bit child mask each, and their leaves stored contiguously in Morton
// order, so a leaf's row is brick_row + popcount(mask bits below its bit).
#include "device_util.h"
#include "internal.h"

namespace art {

__global__ void k_zero_masks(uint32_t* __restrict__ mask, size_t mask_stride,
                             const PoseCounters* __restrict__ cnt) {
    mask += (size_t)blockIdx.y * mask_stride;
    const size_t total = (size_t)cnt[blockIdx.y].nb * 16;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x)
        mask[i] = 0u;
}

// ---------------------------------------------------------------------------
// The skinning has marked every posed brick (key >> 9)
// in a bitmap over the whole brick lattice (2^(3(D+1)-9) bits: 256 KB per pose
// at D = 9), so numbering the occupied bricks in Morton order is a scan of the
// bitmap, and a brick's index is the popcount of the bitmap below its bit:
//   k_dense_bcount, k_dense_bricks : bricks before each bitmap word, the
//                    brick keys in order, nb
//   k_zero_masks   : clear the nb masks
//   k_dense_cells  : per leaf: OR its posed cell's bit into its brick's mask
//                    (one atomic per run of lanes with the same mask word)
//   k_dense_rows   : per pose, one workgroup: brick_row = running sum of the
//                    mask popcounts, M
//   k_dense_place  : per leaf: row = brick_row + mask bits below the cell;
//                    plain stores of the key and the leaf id (one of the
//                    colliding leaves lands), the row kept per leaf
//   k_dense_min    : per leaf: atomicMin on its row when its id is smaller
//                    than the one stored, so the smallest leaf id wins
// ---------------------------------------------------------------------------
__device__ inline uint32_t brick_rank(const uint32_t* __restrict__ bmap, const uint32_t* __restrict__ wpref,
                                      uint32_t brick) {
    const uint32_t w = brick >> 5;
    return wpref[w] + (uint32_t)__popc(bmap[w] & ((1u << (brick & 31u)) - 1u));
}

// The bricks are numbered in two launches over workgroups of 1,024 bitmap
// words each (64 per pose at depth 9): bricks per workgroup, then each
// workgroup adds the counts of the ones before it and numbers its own.
constexpr uint32_t kBrickWordsPerBlock = 1024;

__global__ __launch_bounds__(256) void k_dense_bcount(const uint32_t* __restrict__ bmap, uint32_t bwords,
                                                      uint32_t* __restrict__ blkcnt, uint32_t blk_stride) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const size_t p = blockIdx.y;
    bmap += p * bwords;
    const uint32_t w0 = blockIdx.x * kBrickWordsPerBlock + threadIdx.x * 4u;
    uint32_t c = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
        if (w0 + k < bwords) c += (uint32_t)__popc(bmap[w0 + k]);
    uint32_t tot;
    (void)block_exclusive_scan<256>(c, tmp, &tot);
    if (threadIdx.x == 0) blkcnt[p * blk_stride + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_dense_bricks(const uint32_t* __restrict__ bmap,
                                                      uint32_t* __restrict__ wpref, uint32_t bwords,
                                                      const uint32_t* __restrict__ blkcnt, uint32_t blk_stride,
                                                      uint32_t* __restrict__ brick_key, size_t key_stride,
                                                      PoseCounters* __restrict__ cnt) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const size_t p = blockIdx.y;
    bmap += p * bwords;
    wpref += p * bwords;
    brick_key += p * key_stride;
    blkcnt += p * blk_stride;
    // bricks of the workgroups before this one (gridDim.x <= 256)
    uint32_t before;
    (void)block_exclusive_scan<256>(threadIdx.x < blockIdx.x ? blkcnt[threadIdx.x] : 0u, tmp, &before);
    const uint32_t w0 = blockIdx.x * kBrickWordsPerBlock + threadIdx.x * 4u;
    uint32_t m[4];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        m[k] = w0 + k < bwords ? bmap[w0 + k] : 0u;
        c += (uint32_t)__popc(m[k]);
    }
    uint32_t tot;
    uint32_t base = before + block_exclusive_scan<256>(c, tmp, &tot);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        if (w0 + k >= bwords) break;
        wpref[w0 + k] = base;
        uint32_t v = m[k];
        while (v) {
            const uint32_t b = (uint32_t)__ffs(v) - 1u;
            v &= v - 1u;
            brick_key[base++] = (w0 + k) * 32u + b;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) cnt[p].nb = before + tot;
}

__global__ __launch_bounds__(256) void k_dense_cells(const uint32_t* __restrict__ keys, uint32_t n,
                                                     const uint32_t* __restrict__ bmap,
                                                     const uint32_t* __restrict__ wpref, uint32_t bwords,
                                                     uint32_t* __restrict__ mask) {
    __shared__ LdsOrTable<1024> tab;   // mask words (cell key >> 5) touched by this workgroup
    const size_t p = blockIdx.y;
    keys += p * n;
    bmap += p * bwords;
    wpref += p * bwords;
    mask += p * n * 16;
    tab.init();
    __syncthreads();
    const int lane = lane_id();
    // a contiguous range of leaves per workgroup, four rows of 256 leaves per
    // step with their keys loaded together; lanes past the range hold no key
    // (those with a key are a prefix of the wave)
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, 256, &lo, &hi);
    constexpr uint32_t kRows = 4;
    for (uint32_t base0 = lo; base0 < hi; base0 += kRows * blockDim.x) {
        uint32_t kk[kRows];
#pragma unroll
        for (uint32_t u = 0; u < kRows; ++u) {
            const uint32_t i = base0 + u * blockDim.x + threadIdx.x;
            kk[u] = i < hi ? keys[i] : kInvalidKey;
        }
#pragma unroll
        for (uint32_t u = 0; u < kRows; ++u) {
            const uint32_t base = base0 + u * blockDim.x;
            if (base >= hi) break;   // uniform over the workgroup
            const uint32_t i = base + threadIdx.x;
            const uint32_t key = kk[u];
            const bool ok = key != kInvalidKey;
            // cells share a mask word iff their keys agree above the low 5 bits
            const uint32_t wk = ok ? key >> 5 : kInvalidKey;
            uint32_t bits = ok ? 1u << (key & 31u) : 0u;
            // OR the bits of the following lanes with the same word into each
            // lane; the first lane of every run then holds the run's bits
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t ob = __shfl_down(bits, d, kWave);
                const uint32_t ow = __shfl_down(wk, d, kWave);
                if (lane + d < kWave && i + (uint32_t)d < hi && ow == wk) bits |= ob;
            }
            const uint32_t prev = __shfl_up(wk, 1, kWave);
            if (ok && (lane == 0 || prev != wk) && !tab.insert(wk, bits))
                atomicOr(&mask[(size_t)brick_rank(bmap, wpref, wk >> 4) * 16 + (wk & 15u)], bits);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
        const uint32_t wk = tab.key[e];
        if (wk != kInvalidKey) atomicOr(&mask[(size_t)brick_rank(bmap, wpref, wk >> 4) * 16 + (wk & 15u)], tab.bits[e]);
    }
}

__global__ __launch_bounds__(1024) void k_dense_rows(const uint32_t* __restrict__ mask, size_t n,
                                                     uint32_t* __restrict__ brick_row,
                                                     PoseCounters* __restrict__ cnt) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const size_t p = blockIdx.x;
    mask += p * n * 16;
    brick_row += p * (n + 1);
    const uint32_t nb = cnt[p].nb;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 1024u) {
        const uint32_t b = b0 + threadIdx.x;
        uint32_t c = 0;
        if (b < nb) {
            const uint4* m = reinterpret_cast<const uint4*>(mask + (size_t)b * 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = m[q];
                c += (uint32_t)(__popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w));
            }
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<1024>(c, tmp, &tot);
        if (b < nb) brick_row[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        brick_row[nb] = carry;   // sentinel: end of the last brick
        cnt[p].M = carry;
    }
}

// The per-leaf passes below take 4 leaves per thread, 256 apart, so that each
// thread has 4 independent chains of dependent loads in flight.
constexpr uint32_t kLeafUnroll = 4;   // 8 measured the same or slower

__global__ __launch_bounds__(256) void k_dense_place(const uint32_t* __restrict__ keys, uint32_t n,
                                                     const uint32_t* __restrict__ bmap,
                                                     const uint32_t* __restrict__ wpref, uint32_t bwords,
                                                     const uint32_t* __restrict__ mask,
                                                     const uint32_t* __restrict__ brick_row,
                                                     uint32_t* __restrict__ occ_key, uint32_t* __restrict__ occ_win,
                                                     uint32_t* __restrict__ rows) {
    const size_t p = blockIdx.y;
    keys += p * n;
    bmap += p * bwords;
    wpref += p * bwords;
    mask += p * n * 16;
    brick_row += p * (n + 1);
    if (occ_key) occ_key += p * n;
    occ_win += p * n;
    rows += p * n;
    const uint32_t step = gridDim.x * blockDim.x * kLeafUnroll;
    for (uint32_t base = blockIdx.x * blockDim.x * kLeafUnroll + threadIdx.x; base < n; base += step) {
        uint32_t key[kLeafUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kLeafUnroll; ++u) {
            const uint32_t i = base + u * blockDim.x;
            key[u] = i < n ? keys[i] : kInvalidKey;
        }
#pragma unroll
        for (uint32_t u = 0; u < kLeafUnroll; ++u) {
            const uint32_t i = base + u * blockDim.x;
            uint32_t row = kInvalidKey;
            if (key[u] != kInvalidKey) {
                const uint32_t bi = brick_rank(bmap, wpref, key[u] >> 9);
                const uint32_t local = key[u] & 511u;
                const uint32_t wsel = local >> 5;
                const uint4* m = reinterpret_cast<const uint4*>(mask + (size_t)bi * 16);
                uint32_t below = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint4 v = m[q];
                    const uint32_t mw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t j = (uint32_t)(4 * q + e);
                        const uint32_t part =
                            j < wsel ? mw[e] : (j == wsel ? mw[e] & ((1u << (local & 31u)) - 1u) : 0u);
                        below += (uint32_t)__popc(part);
                    }
                }
                row = brick_row[bi] + below;
                if (occ_key) occ_key[row] = key[u];
                occ_win[row] = i;
            }
            if (i < n) rows[i] = row;
        }
    }
}

__global__ __launch_bounds__(256) void k_dense_min(const uint32_t* __restrict__ rows, uint32_t n,
                                                   uint32_t* __restrict__ occ_win) {
    const size_t p = blockIdx.y;
    rows += p * n;
    occ_win += p * n;
    const uint32_t step = gridDim.x * blockDim.x * kLeafUnroll;
    for (uint32_t base = blockIdx.x * blockDim.x * kLeafUnroll + threadIdx.x; base < n; base += step) {
        uint32_t row[kLeafUnroll], cur[kLeafUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kLeafUnroll; ++u) {
            const uint32_t i = base + u * blockDim.x;
            row[u] = i < n ? rows[i] : kInvalidKey;
        }
#pragma unroll
        for (uint32_t u = 0; u < kLeafUnroll; ++u) cur[u] = row[u] != kInvalidKey ? occ_win[row[u]] : 0u;
        // the stored id only decreases, so a stale read can only cause an extra atomic
#pragma unroll
        for (uint32_t u = 0; u < kLeafUnroll; ++u) {
            const uint32_t i = base + u * blockDim.x;
            if (row[u] != kInvalidKey && i < cur[u]) atomicMin(&occ_win[row[u]], i);
        }
    }
}

hipError_t launch_build_octree_dense(const uint32_t* keys, uint32_t n, int depth, Scratch& s, const OctreeSlot& o,
                                     int batch, hipStream_t st, int* launches) {
    PoseCounters* cnt = s.counters.as<PoseCounters>();
    const uint32_t bwords = brick_words(depth);
    uint32_t* bmap = s.bmap.as<uint32_t>();
    uint32_t* wpref = s.wpref.as<uint32_t>();
    uint32_t* rows = s.keys1.as<uint32_t>();   // [batch][n] posed row of each leaf
    int grid = (int)((n + 255) / 256);
    if (grid > 2048) grid = 2048;
    const uint32_t nbw = (bwords + kBrickWordsPerBlock - 1) / kBrickWordsPerBlock;   // <= 64 (depth <= 9)
    if (nbw > 256 || nbw > (uint32_t)kUniqueBlocks) return hipErrorInvalidValue;
    uint32_t* blkcnt = s.blk1.as<uint32_t>();   // [batch][kUniqueBlocks]
    hipLaunchKernelGGL(k_dense_bcount, dim3(nbw, batch), dim3(256), 0, st, (const uint32_t*)bmap, bwords, blkcnt,
                       (uint32_t)kUniqueBlocks);
    hipLaunchKernelGGL(k_dense_bricks, dim3(nbw, batch), dim3(256), 0, st, (const uint32_t*)bmap, wpref, bwords,
                       (const uint32_t*)blkcnt, (uint32_t)kUniqueBlocks, o.brick_key, (size_t)n, cnt);
    hipLaunchKernelGGL(k_zero_masks, dim3(256, batch), dim3(256), 0, st, o.brick_mask, (size_t)n * 16,
                       (const PoseCounters*)cnt);
    const int cgrid = std::min(grid, 512);   // ~3k leaves per workgroup at 1.5M leaves
    hipLaunchKernelGGL(k_dense_cells, dim3(cgrid, batch), dim3(256), 0, st, keys, n, (const uint32_t*)bmap,
                       (const uint32_t*)wpref, bwords, o.brick_mask);
    hipLaunchKernelGGL(k_dense_rows, dim3(batch), dim3(1024), 0, st, (const uint32_t*)o.brick_mask, (size_t)n,
                       o.brick_row, cnt);
    const int lgrid = (int)std::min<uint32_t>((n + 256 * kLeafUnroll - 1) / (256 * kLeafUnroll), 2048u);
    hipLaunchKernelGGL(k_dense_place, dim3(lgrid, batch), dim3(256), 0, st, keys, n, (const uint32_t*)bmap,
                       (const uint32_t*)wpref, bwords, (const uint32_t*)o.brick_mask,
                       (const uint32_t*)o.brick_row, o.occ_key, o.occ_win, rows);
    hipLaunchKernelGGL(k_dense_min, dim3(lgrid, batch), dim3(256), 0, st, (const uint32_t*)rows, n, o.occ_win);
    *launches += 7;
    return hipGetLastError();
}

}  // namespace art
