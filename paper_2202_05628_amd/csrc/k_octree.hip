// Posed-octree rebuild after the key sort (Section 3.1: the octree is rebuilt
// for every pose; leaves warped onto one cell collide and one of them is kept).
//
// Input: posed Morton keys sorted stably with the canonical leaf id as payload,
// so within a run of equal keys the first payload is the smallest leaf id -
// the collision winner.  Dropped leaves carry the invalid key and sort last.
//
//   k_unique_count : per block, count cell-run starts, brick-run starts
//                    (key >> 9 changes) and dropped leaves
//   k_unique_scan  : one workgroup scans the block counts -> M, nb
//   k_zero_masks   : clear the 512-bit occupancy masks of the nb bricks
//   k_unique_write : per cell run: occupied key, winner id and the cell's bit
//                    in its brick mask; per brick run: brick key and first row.
//
// The result is a two-level octree: bricks (the level 3 above the leaves) with
// a 512-bit child mask each, and their leaves stored contiguously in Morton
// order, so a leaf's row is brick_row + popcount(mask bits below its bit).
#include "device_util.h"
#include "internal.h"

namespace art {

constexpr int kUThreads = 256;

__global__ __launch_bounds__(kUThreads) void k_unique_count(const uint32_t* __restrict__ skeys,
                                                            uint32_t n,
                                                            uint32_t* __restrict__ blk_run,
                                                            uint32_t* __restrict__ blk_brick,
                                                            PoseCounters* __restrict__ cnt) {
    __shared__ uint32_t sr[kUThreads / kWave], sb[kUThreads / kWave], sd[kUThreads / kWave];
    const uint32_t p = blockIdx.y;
    skeys += (size_t)p * n;
    blk_run += (size_t)p * gridDim.x;
    blk_brick += (size_t)p * gridDim.x;
    cnt += p;
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, kUThreads, &lo, &hi);
    uint32_t nr = 0, nbk = 0, nd = 0;   // (same block ranges as k_unique_write)
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kUThreads) {
        const uint32_t k = skeys[i];
        const uint32_t kp = i > 0 ? skeys[i - 1] : kInvalidKey;
        const bool valid = k != kInvalidKey;
        nr += (valid && (i == 0 || kp != k)) ? 1u : 0u;
        nbk += (valid && (i == 0 || (kp >> 9) != (k >> 9))) ? 1u : 0u;
        nd += valid ? 0u : 1u;
    }
    nr = wave_sum(nr);
    nbk = wave_sum(nbk);
    nd = wave_sum(nd);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        sr[w] = nr;
        sb[w] = nbk;
        sd[w] = nd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0, c = 0;
        for (int q = 0; q < kUThreads / kWave; ++q) {
            a += sr[q];
            b += sb[q];
            c += sd[q];
        }
        blk_run[blockIdx.x] = a;
        blk_brick[blockIdx.x] = b;
        if (c) atomicAdd(&cnt->dropped, c);
    }
}

__global__ __launch_bounds__(1024) void k_unique_scan(uint32_t* __restrict__ blk_run,
                                                      uint32_t* __restrict__ blk_brick, int nblk,
                                                      PoseCounters* __restrict__ cnt,
                                                      uint32_t* __restrict__ brick_row, size_t row_stride) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const uint32_t p = blockIdx.x;
    blk_run += (size_t)p * nblk;
    blk_brick += (size_t)p * nblk;
    cnt += p;
    brick_row += p * row_stride;
    const int t = threadIdx.x;
    uint32_t a = t < nblk ? blk_run[t] : 0u;
    uint32_t ta;
    uint32_t ea = block_exclusive_scan<1024>(a, tmp, &ta);
    uint32_t b = t < nblk ? blk_brick[t] : 0u;
    uint32_t tb;
    uint32_t eb = block_exclusive_scan<1024>(b, tmp, &tb);
    if (t < nblk) {
        blk_run[t] = ea;
        blk_brick[t] = eb;
    }
    if (t == 0) {
        cnt->M = ta;
        cnt->nb = tb;
        brick_row[tb] = ta;   // sentinel: end of the last brick
    }
}

__global__ void k_zero_masks(uint32_t* __restrict__ mask, size_t mask_stride,
                             const PoseCounters* __restrict__ cnt) {
    mask += (size_t)blockIdx.y * mask_stride;
    const size_t total = (size_t)cnt[blockIdx.y].nb * 16;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x)
        mask[i] = 0u;
}

// Each thread owns kUItems consecutive sorted keys; one block scan of the
// packed (cell runs | brick runs << 16) counts per 256 * kUItems keys.
constexpr int kUItems = 8;

__global__ __launch_bounds__(kUThreads) void k_unique_write(
    const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ svals, uint32_t n,
    const uint32_t* __restrict__ blk_run, const uint32_t* __restrict__ blk_brick,
    uint32_t* __restrict__ occ_key, uint32_t* __restrict__ occ_win,
    uint32_t* __restrict__ brick_key, uint32_t* __restrict__ brick_row,
    uint32_t* __restrict__ brick_mask) {
    __shared__ uint32_t tmp[kUThreads / kWave + 1];
    const size_t p = blockIdx.y;
    skeys += p * n;
    svals += p * n;
    blk_run += p * gridDim.x;
    blk_brick += p * gridDim.x;
    occ_key += p * n;
    occ_win += p * n;
    brick_key += p * n;
    brick_row += p * (n + 1);
    brick_mask += p * n * 16;
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, kUThreads, &lo, &hi);
    uint32_t carry_r = blk_run[blockIdx.x];
    uint32_t carry_b = blk_brick[blockIdx.x];
    for (uint32_t t0 = lo; t0 < hi; t0 += kUThreads * kUItems) {
        const uint32_t i0 = t0 + threadIdx.x * kUItems;
        uint32_t k[kUItems];
        uint32_t prev = (i0 > 0 && i0 - 1 < hi) ? skeys[i0 - 1] : kInvalidKey;
        uint32_t flags = 0;   // bit j: cell run start, bit 8 + j: brick run start
        uint32_t nr = 0, nbk = 0;
#pragma unroll
        for (int j = 0; j < kUItems; ++j) {
            const uint32_t i = i0 + j;
            k[j] = i < hi ? skeys[i] : kInvalidKey;
            const bool valid = k[j] != kInvalidKey;
            const bool rs = valid && (i == 0 || prev != k[j]);
            const bool bs = valid && (i == 0 || (prev >> 9) != (k[j] >> 9));
            flags |= (rs ? 1u : 0u) << j;
            flags |= (bs ? 1u : 0u) << (8 + j);
            nr += rs ? 1u : 0u;
            nbk += bs ? 1u : 0u;
            prev = k[j];
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<kUThreads>(nr | (nbk << 16), tmp, &tot);
        uint32_t m = carry_r + (ex & 0xFFFFu);
        uint32_t bc = carry_b + (ex >> 16);   // bricks started before this thread's items
        // Cells of one mask word are consecutive in Morton order: their bits are
        // gathered in a register and OR-ed into the word once per run (words
        // shared with a neighbouring thread's items still meet in the atomic).
        size_t word = ~(size_t)0;
        uint32_t bits = 0;
#pragma unroll
        for (int j = 0; j < kUItems; ++j) {
            const bool rs = (flags >> j) & 1u;
            const bool bs = (flags >> (8 + j)) & 1u;
            if (bs) {
                brick_key[bc] = k[j] >> 9;
                brick_row[bc] = m;
                ++bc;
            }
            if (rs) {
                const uint32_t id = svals[i0 + j];
                occ_key[m] = k[j];
                occ_win[m] = id;
                const uint32_t local = k[j] & 511u;
                const size_t wi = (size_t)(bc - 1) * 16 + (local >> 5);
                if (wi != word) {
                    if (bits) atomicOr(&brick_mask[word], bits);
                    word = wi;
                    bits = 0;
                }
                bits |= 1u << (local & 31u);
                ++m;
            }
        }
        if (bits) atomicOr(&brick_mask[word], bits);
        carry_r += tot & 0xFFFFu;
        carry_b += tot >> 16;
    }
}

hipError_t launch_build_octree(const uint32_t* skeys, const uint32_t* svals, uint32_t n, Scratch& s,
                               const OctreeSlot& o, int batch, hipStream_t st, int* launches) {
    PoseCounters* cnt = s.counters.as<PoseCounters>();
    hipLaunchKernelGGL(k_unique_count, dim3(kUniqueBlocks, batch), dim3(kUThreads), 0, st, skeys, n,
                       s.blk0.as<uint32_t>(), s.blk1.as<uint32_t>(), cnt);
    hipLaunchKernelGGL(k_unique_scan, dim3(batch), dim3(1024), 0, st, s.blk0.as<uint32_t>(), s.blk1.as<uint32_t>(),
                       kUniqueBlocks, cnt, o.brick_row, (size_t)n + 1);
    hipLaunchKernelGGL(k_zero_masks, dim3(256, batch), dim3(256), 0, st, o.brick_mask, (size_t)n * 16,
                       (const PoseCounters*)cnt);
    hipLaunchKernelGGL(k_unique_write, dim3(kUniqueBlocks, batch), dim3(kUThreads), 0, st, skeys, svals, n,
                       s.blk0.as<uint32_t>(), s.blk1.as<uint32_t>(), o.occ_key, o.occ_win, o.brick_key, o.brick_row,
                       o.brick_mask);
    *launches += 4;
    return hipGetLastError();
}

}  // namespace art
