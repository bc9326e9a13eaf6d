// Device helpers shared by the renderer's HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace art {

constexpr int kWave = 64;
constexpr uint32_t kInvalidKey = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Morton codes: x in the lowest bit of each 3-bit group
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}
__host__ __device__ inline uint32_t compact2(uint32_t v) {   // even bits -> low half
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ inline uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Make LDS writes of this wave visible to its other lanes.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline T wave_inclusive_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (l >= d) v += u;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Block-wide exclusive scan for blockDim.x == NT (multiple of 64, <= 1024).
// `tmp` is LDS of at least NT/64 + 1 elements.  Returns the exclusive prefix
// and writes the block total to *total.  Contains __syncthreads.
template <int NT, typename T>
__device__ inline T block_exclusive_scan(T v, T* tmp, T* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane_id() == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (w == 0) {
        T s = lane_id() < NW ? tmp[lane_id()] : T(0);
        T si = wave_inclusive_scan(s);
        if (lane_id() < NW) tmp[lane_id()] = si - s;
        if (lane_id() == NW - 1) tmp[NW] = si;
    }
    __syncthreads();
    T out = tmp[w] + inc - v;
    *total = tmp[NW];
    __syncthreads();
    return out;
}

// Contiguous range of `n` items owned by block `b` of `nb` blocks (tile aligned).
__device__ inline void block_range(uint32_t n, uint32_t b, uint32_t nb, uint32_t align,
                                   uint32_t* lo, uint32_t* hi) {
    uint32_t per = (n + nb - 1) / nb;
    per = (per + align - 1) / align * align;
    uint64_t l = (uint64_t)b * per;
    uint64_t h = l + per;
    *lo = (uint32_t)(l < n ? l : n);
    *hi = (uint32_t)(h < n ? h : n);
}

// Streaming stores of output maps, which nothing reads again in the same
// launch: non-temporal, so they do not displace the gathered FLUT rows and
// octree lines from the caches.
#ifndef ART_NT_STORES
#define ART_NT_STORES 1
#endif
typedef float art_f4 __attribute__((ext_vector_type(4)));
__device__ inline void store_stream(float* p, float v) {
#if ART_NT_STORES
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}
__device__ inline void store_stream4(float* p, float4 v) {   // p 16-byte aligned
    const art_f4 w = {v.x, v.y, v.z, v.w};
#if ART_NT_STORES
    __builtin_nontemporal_store(w, reinterpret_cast<art_f4*>(p));
#else
    *reinterpret_cast<art_f4*>(p) = w;
#endif
}

// Workgroup-local merging of OR-updates to 32-bit words named by a key (any
// value but kInvalidKey): an open-addressing table of N entries (a power of
// two) in LDS, so that each distinct key costs one global atomic per
// workgroup instead of one per update.
template <int N>
struct LdsOrTable {
    uint32_t key[N];
    uint32_t bits[N];
    __device__ void init() {
        for (int e = threadIdx.x; e < N; e += blockDim.x) {
            key[e] = kInvalidKey;
            bits[e] = 0u;
        }
    }
    // false when the table is full: the caller then updates the global word itself
    __device__ bool insert(uint32_t k, uint32_t b) {
        static_assert((N & (N - 1)) == 0, "N must be a power of two");
        uint32_t h = (k * 0x9E3779B1u) >> (32 - __builtin_ctz(N));
        for (int probe = 0; probe < N; ++probe) {
            const uint32_t old = atomicCAS(&key[h], kInvalidKey, k);
            if (old == kInvalidKey || old == k) {
                atomicOr(&bits[h], b);
                return true;
            }
            h = (h + 1u) & (uint32_t)(N - 1);
        }
        return false;
    }
};

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Rotation matrix (row-major 3x3) of an axis-angle vector r, FP64 (Rodrigues).
__device__ inline void axis_angle_to_matrix(const double* r, double* M) {
    const double t2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double t = sqrt(t2);
    if (t < 1e-12) {
        M[0] = 1; M[1] = 0; M[2] = 0;
        M[3] = 0; M[4] = 1; M[5] = 0;
        M[6] = 0; M[7] = 0; M[8] = 1;
        return;
    }
    const double kx = r[0] / t, ky = r[1] / t, kz = r[2] / t;
    double s, c;
    sincos(t, &s, &c);
    const double v = 1.0 - c;
    // R = c I + s [k]_x + (1 - c) k k^T
    M[0] = c + v * kx * kx;      M[1] = v * kx * ky - s * kz; M[2] = v * kx * kz + s * ky;
    M[3] = v * ky * kx + s * kz; M[4] = c + v * ky * ky;      M[5] = v * ky * kz - s * kx;
    M[6] = v * kz * kx - s * ky; M[7] = v * kz * ky + s * kx; M[8] = c + v * kz * kz;
}


}  // namespace art
