// Data-parallel primitives of the posed-octree rebuild, batched over the poses
// of a launch (pose = blockIdx.y): a stable LSD radix sort of (uint32 key,
// uint32 payload) pairs and an exclusive scan.  Every kernel has a fixed grid;
// the item count of each pose is read from device memory, so the host never
// waits for a count produced on the GPU.
//
// Radix pass (8-bit digit, blocks own contiguous key ranges of their pose):
//   k_hist     per-block digit histogram           -> hist[pose][digit][block]
//   k_hscan    one wave per (digit, pose) scans its row over the blocks
//              and writes the digit total
//   k_scatter  per block, tiles of 4096 keys staged in LDS in stable digit
//              order (lanes with equal digits matched with 8 wave ballots and
//              ranked by lane; waves and 256-key sub-tiles ordered through LDS
//              counters), then written digit run by digit run.
#include "device_util.h"
#include "internal.h"

namespace art {

constexpr int kSortThreads = 256;

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(kSortThreads) void k_hist(const uint32_t* __restrict__ keys, size_t kstride,
                                                       const uint32_t* __restrict__ d_n, uint32_t nstride,
                                                       int shift, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    const uint32_t p = blockIdx.y;
    keys += p * kstride;
    hist += (size_t)p * 256 * gridDim.x;
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t lo, hi;
    block_range(d_n[p * nstride], blockIdx.x, gridDim.x, kSortThreads, &lo, &hi);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kSortThreads)
        atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// One wave per (digit, pose), nblk <= 512: each lane takes 8 consecutive
// blocks of the digit's row (a serial prefix), the lanes' sums are scanned
// across the wave.
constexpr int kHscanPerLane = 8;
static_assert(kSortBlocks <= kWave * kHscanPerLane, "one wave scans a digit's row");
__global__ __launch_bounds__(kWave) void k_hscan(uint32_t* __restrict__ hist, int nblk,
                                                 uint32_t* __restrict__ digit_tot) {
    const int d = blockIdx.x;
    const uint32_t p = blockIdx.y;
    uint32_t* row = hist + ((size_t)p * 256 + d) * nblk;
    const int lane = threadIdx.x;
    uint32_t v[kHscanPerLane];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kHscanPerLane; ++j) {
        const int b = kHscanPerLane * lane + j;
        v[j] = b < nblk ? row[b] : 0u;
        sum += v[j];
    }
    const uint32_t incl = wave_inclusive_scan(sum);
    uint32_t run = incl - sum;
#pragma unroll
    for (int j = 0; j < kHscanPerLane; ++j) {
        const int b = kHscanPerLane * lane + j;
        if (b < nblk) row[b] = run;
        run += v[j];
    }
    if (lane == kWave - 1) digit_tot[(size_t)p * 256 + d] = incl;
}

// Keys per block iteration of the scatter: 16 sub-tiles of 256.
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

// Stable scatter of one digit pass.  A block stages each tile of 4096 keys in
// LDS in digit order (stable ranks: lanes with equal digits are matched with 8
// wave ballots and ranked by lane; waves and sub-tiles are ordered through LDS
// counters), then writes the tile digit run by digit run, so consecutive
// threads store to consecutive addresses of a run.
__global__ __launch_bounds__(kSortThreads) void k_scatter(
    const uint32_t* __restrict__ kin, uint32_t* __restrict__ kout, size_t kstride,
    const uint32_t* __restrict__ vin, uint32_t* __restrict__ vout, size_t vstride,
    const uint32_t* __restrict__ d_n, uint32_t nstride, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ digit_tot) {
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t base[256];     // next global position of each digit for this block
    __shared__ uint32_t lstart[256];   // first staged slot of each digit in the tile
    __shared__ uint32_t lcount[256];   // keys of each digit in the tile
    __shared__ uint32_t run[256];      // keys of each digit staged so far
    __shared__ uint32_t cnt[NW][256];  // per-wave digit counts of the current sub-tile
    __shared__ uint32_t tmp[NW + 1];
    __shared__ uint32_t sk[kSortTile];
    __shared__ uint32_t sv[kSortTile];
    const uint32_t p = blockIdx.y;
    kin += p * kstride;
    kout += p * kstride;
    vin += p * vstride;
    vout += p * vstride;
    hist += (size_t)p * 256 * gridDim.x;
    digit_tot += (size_t)p * 256;
    const int t = threadIdx.x;
    const int w = t / kWave;
    uint32_t tot;
    const uint32_t dpre = block_exclusive_scan<kSortThreads>(digit_tot[t], tmp, &tot);
    base[t] = dpre + hist[t * gridDim.x + blockIdx.x];
#pragma unroll
    for (int q = 0; q < NW; ++q) cnt[q][t] = 0;
    uint32_t lo, hi;
    block_range(d_n[p * nstride], blockIdx.x, gridDim.x, kSortThreads, &lo, &hi);
    const uint64_t below = lanemask_lt();
    for (uint32_t i0 = lo; i0 < hi; i0 += kSortTile) {
        const uint32_t m = (hi - i0) < (uint32_t)kSortTile ? (hi - i0) : (uint32_t)kSortTile;
        lcount[t] = 0;
        run[t] = 0;
        __syncthreads();
        uint32_t k[kSortItems], v[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const uint32_t idx = (uint32_t)(j * kSortThreads + t);
            const bool valid = idx < m;
            k[j] = valid ? kin[i0 + idx] : 0u;
            v[j] = valid ? vin[i0 + idx] : 0u;
            if (valid) atomicAdd(&lcount[(k[j] >> shift) & 255u], 1u);
        }
        __syncthreads();
        uint32_t ttot;
        lstart[t] = block_exclusive_scan<kSortThreads>(lcount[t], tmp, &ttot);
        __syncthreads();
        // stable staging, sub-tile by sub-tile
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if ((uint32_t)(j * kSortThreads) >= m) break;   // uniform over the block
            const bool valid = (uint32_t)(j * kSortThreads + t) < m;
            const uint32_t d = (k[j] >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) {
                const bool bit = (d >> bb) & 1u;
                const uint64_t mm = __ballot(bit);
                peers &= bit ? mm : ~mm;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & below);
            if (valid && rank == 0) cnt[w][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t pre = run[d] + rank;
                for (int q = 0; q < w; ++q) pre += cnt[q][d];
                const uint32_t slot = lstart[d] + pre;
                sk[slot] = k[j];
                sv[slot] = v[j];
            }
            __syncthreads();
            uint32_t add = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                add += cnt[q][t];
                cnt[q][t] = 0;
            }
            run[t] += add;
            __syncthreads();
        }
        // write the staged tile run by run
        for (uint32_t e = (uint32_t)t; e < m; e += kSortThreads) {
            const uint32_t key = sk[e];
            const uint32_t d = (key >> shift) & 255u;
            const uint32_t dst = base[d] + (e - lstart[d]);
            kout[dst] = key;
            vout[dst] = sv[e];
        }
        __syncthreads();
        base[t] += lcount[t];
        __syncthreads();
    }
}

hipError_t launch_radix_sort(const SortBatch& b, int bits, hipStream_t st, bool* result_in_1, int* launches) {
    int nblk = (int)((b.n_cap + kSortTile - 1) / kSortTile);
    if (nblk < 1) nblk = 1;
    if (nblk > kSortBlocks) nblk = kSortBlocks;
    const int passes = (bits + 7) / 8;
    uint32_t *ki = b.k0, *vi = b.v0, *ko = b.k1, *vo = b.v1;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_hist, dim3(nblk, b.batch), dim3(kSortThreads), 0, st, ki, b.kstride, b.d_n, b.nstride,
                           shift, b.hist);
        hipLaunchKernelGGL(k_hscan, dim3(256, b.batch), dim3(kWave), 0, st, b.hist, nblk, b.digit_tot);
        hipLaunchKernelGGL(k_scatter, dim3(nblk, b.batch), dim3(kSortThreads), 0, st, ki, ko, b.kstride, vi, vo,
                           b.vstride, b.d_n, b.nstride, shift, b.hist, b.digit_tot);
        *launches += 3;
        uint32_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    *result_in_1 = (passes & 1) != 0;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of a device-sized uint32 array per pose
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, size_t stride,
                                                              const uint32_t* __restrict__ d_n, uint32_t nstride,
                                                              uint32_t* __restrict__ blk) {
    __shared__ uint32_t tmp[kScanThreads / kWave];
    const uint32_t p = blockIdx.y;
    in += p * stride;
    blk += (size_t)p * gridDim.x;
    uint32_t lo, hi;
    block_range(d_n[p * nstride], blockIdx.x, gridDim.x, kScanThreads, &lo, &hi);
    uint32_t s = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kScanThreads) s += in[i];
    s = wave_sum(s);
    if (lane_id() == 0) tmp[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int q = 0; q < kScanThreads / kWave; ++q) t += tmp[q];
        blk[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* __restrict__ blk, int nblk,
                                                      uint32_t* __restrict__ d_total, uint32_t tstride) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const uint32_t p = blockIdx.x;
    blk += (size_t)p * nblk;
    uint32_t v = (int)threadIdx.x < nblk ? blk[threadIdx.x] : 0u;
    uint32_t total;
    uint32_t ex = block_exclusive_scan<1024>(v, tmp, &total);
    if ((int)threadIdx.x < nblk) blk[threadIdx.x] = ex;
    if (threadIdx.x == 0 && d_total) d_total[p * tstride] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ in,
                                                            uint32_t* __restrict__ out, size_t stride,
                                                            const uint32_t* __restrict__ d_n, uint32_t nstride,
                                                            const uint32_t* __restrict__ blk) {
    __shared__ uint32_t tmp[kScanThreads / kWave + 1];
    const uint32_t p = blockIdx.y;
    in += p * stride;
    out += p * stride;
    uint32_t lo, hi;
    block_range(d_n[p * nstride], blockIdx.x, gridDim.x, kScanThreads, &lo, &hi);
    uint32_t carry = blk[(size_t)p * gridDim.x + blockIdx.x];
    for (uint32_t i0 = lo; i0 < hi; i0 += kScanThreads) {
        const uint32_t i = i0 + threadIdx.x;
        const uint32_t v = i < hi ? in[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<kScanThreads>(v, tmp, &total);
        if (i < hi) out[i] = carry + ex;
        carry += total;
    }
}

hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, size_t stride, const uint32_t* d_n,
                                 uint32_t nstride, uint32_t* d_total, uint32_t tstride, uint32_t* blk, int batch,
                                 hipStream_t st, int* launches) {
    const int nblk = kScanBlocks;   // per pose; blk holds batch * nblk partials
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk, batch), dim3(kScanThreads), 0, st, in, stride, d_n, nstride, blk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(batch), dim3(1024), 0, st, blk, nblk, d_total, tstride);
    hipLaunchKernelGGL(k_scan_down, dim3(nblk, batch), dim3(kScanThreads), 0, st, in, out, stride, d_n, nstride,
                       blk);
    *launches += 3;
    return hipGetLastError();
}

}  // namespace art
