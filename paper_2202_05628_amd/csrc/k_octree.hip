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
//   k_unique_write : per cell run: occupied key, winner id, the FLUT row of the
//                    winner copied into posed (Morton) order, the cell's bit in
//                    its brick mask; per brick run: brick key and first row.
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
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, kUThreads, &lo, &hi);
    uint32_t nr = 0, nbk = 0, nd = 0;
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
                                                      uint32_t* __restrict__ brick_row) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
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

__global__ void k_zero_masks(uint32_t* __restrict__ mask, const PoseCounters* __restrict__ cnt) {
    const size_t total = (size_t)cnt->nb * 16;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x)
        mask[i] = 0u;
}

template <int ROW_BYTES, int SIG_BYTES>
__global__ __launch_bounds__(kUThreads) void k_unique_write(
    const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ svals, uint32_t n,
    const uint32_t* __restrict__ blk_run, const uint32_t* __restrict__ blk_brick,
    uint32_t* __restrict__ occ_key, uint32_t* __restrict__ occ_win,
    uint32_t* __restrict__ brick_key, uint32_t* __restrict__ brick_row,
    uint32_t* __restrict__ brick_mask, const uint8_t* __restrict__ sigma,
    const uint8_t* __restrict__ feat, uint8_t* __restrict__ psig, uint8_t* __restrict__ pfeat) {
    __shared__ uint32_t tmp[kUThreads / kWave + 1];
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, kUThreads, &lo, &hi);
    uint32_t carry_r = blk_run[blockIdx.x];
    uint32_t carry_b = blk_brick[blockIdx.x];
    for (uint32_t i0 = lo; i0 < hi; i0 += kUThreads) {
        const uint32_t i = i0 + threadIdx.x;
        uint32_t k = kInvalidKey, kp = kInvalidKey;
        if (i < hi) {
            k = skeys[i];
            kp = i > 0 ? skeys[i - 1] : kInvalidKey;
        }
        const bool valid = k != kInvalidKey;
        const bool rs = valid && (i == 0 || kp != k);
        const bool bs = valid && (i == 0 || (kp >> 9) != (k >> 9));
        uint32_t tr, tb;
        const uint32_t er = block_exclusive_scan<kUThreads>(rs ? 1u : 0u, tmp, &tr);
        const uint32_t eb = block_exclusive_scan<kUThreads>(bs ? 1u : 0u, tmp, &tb);
        const uint32_t m = carry_r + er;
        const uint32_t bi = carry_b + eb + (bs ? 1u : 0u) - 1u;   // brick holding element i
        if (bs) {
            brick_key[bi] = k >> 9;
            brick_row[bi] = m;
        }
        if (rs) {
            const uint32_t id = svals[i];
            occ_key[m] = k;
            occ_win[m] = id;
            const uint32_t local = k & 511u;
            atomicOr(&brick_mask[(size_t)bi * 16 + (local >> 5)], 1u << (local & 31u));
            // winner's FLUT row in posed order
            if (SIG_BYTES == 4)
                reinterpret_cast<uint32_t*>(psig)[m] = reinterpret_cast<const uint32_t*>(sigma)[id];
            else
                reinterpret_cast<uint16_t*>(psig)[m] = reinterpret_cast<const uint16_t*>(sigma)[id];
            if constexpr (ROW_BYTES % 16 == 0) {
                const uint4* src = reinterpret_cast<const uint4*>(feat + (size_t)id * ROW_BYTES);
                uint4* dst = reinterpret_cast<uint4*>(pfeat + (size_t)m * ROW_BYTES);
#pragma unroll
                for (int q = 0; q < ROW_BYTES / 16; ++q) dst[q] = src[q];
            } else {
                const uint2* src = reinterpret_cast<const uint2*>(feat + (size_t)id * ROW_BYTES);
                uint2* dst = reinterpret_cast<uint2*>(pfeat + (size_t)m * ROW_BYTES);
#pragma unroll
                for (int q = 0; q < ROW_BYTES / 8; ++q) dst[q] = src[q];
            }
        }
        carry_r += tr;
        carry_b += tb;
    }
}

template <int ROW_BYTES, int SIG_BYTES>
static void launch_write(const uint32_t* skeys, const uint32_t* svals, uint32_t n, Scratch& s,
                         const OctreeSlot& o, const void* sigma, const void* feat, hipStream_t st) {
    hipLaunchKernelGGL((k_unique_write<ROW_BYTES, SIG_BYTES>), dim3(kUniqueBlocks), dim3(kUThreads),
                       0, st, skeys, svals, n, s.blk0.as<uint32_t>(), s.blk1.as<uint32_t>(), o.occ_key,
                       o.occ_win, o.brick_key, o.brick_row, o.brick_mask,
                       static_cast<const uint8_t*>(sigma), static_cast<const uint8_t*>(feat),
                       static_cast<uint8_t*>(o.psig), static_cast<uint8_t*>(o.pfeat));
}

hipError_t launch_build_octree(const uint32_t* skeys, const uint32_t* svals, uint32_t n, int C,
                               int storage, const void* sigma, const void* feat, Scratch& s,
                               const OctreeSlot& o, hipStream_t st, int* launches) {
    PoseCounters* cnt = s.counters.as<PoseCounters>();
    hipLaunchKernelGGL(k_unique_count, dim3(kUniqueBlocks), dim3(kUThreads), 0, st, skeys, n,
                       s.blk0.as<uint32_t>(), s.blk1.as<uint32_t>(), cnt);
    hipLaunchKernelGGL(k_unique_scan, dim3(1), dim3(1024), 0, st, s.blk0.as<uint32_t>(),
                       s.blk1.as<uint32_t>(), kUniqueBlocks, cnt, o.brick_row);
    hipLaunchKernelGGL(k_zero_masks, dim3(1024), dim3(256), 0, st, o.brick_mask,
                       (const PoseCounters*)cnt);
    *launches += 4;
    const int es = storage == ART_BF16 ? 2 : 4;
    switch (C * es) {
        case 8: launch_write<8, 2>(skeys, svals, n, s, o, sigma, feat, st); break;     // C=4 bf16
        case 16:
            if (es == 4) launch_write<16, 4>(skeys, svals, n, s, o, sigma, feat, st);  // C=4 f32
            else launch_write<16, 2>(skeys, svals, n, s, o, sigma, feat, st);          // C=8 bf16
            break;
        case 32:
            if (es == 4) launch_write<32, 4>(skeys, svals, n, s, o, sigma, feat, st);
            else launch_write<32, 2>(skeys, svals, n, s, o, sigma, feat, st);
            break;
        case 64:
            if (es == 4) launch_write<64, 4>(skeys, svals, n, s, o, sigma, feat, st);
            else launch_write<64, 2>(skeys, svals, n, s, o, sigma, feat, st);
            break;
        case 128: launch_write<128, 4>(skeys, svals, n, s, o, sigma, feat, st); break;  // C=32 f32
        default: return hipErrorInvalidValue;
    }
    *launches += 1;
    return hipGetLastError();
}

}  // namespace art
