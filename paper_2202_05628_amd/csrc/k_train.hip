// Kernels of the FLUT training step (Section 3.1, "Training"):
//
//   k_vrt        : the voxel regularisation term of Eq. 10 for every pose of a
//                  batch and its gradient with respect to the features.
//                  Q(p_i^t, T^t) is the feature of the collision winner of the
//                  posed cell holding leaf i (the row the octree build gave the
//                  leaf); L += lambda / N_v * |f_w - f_i|_1 over the leaves
//                  inside the posed root, and sign(f_w - f_i) * lambda / N_v
//                  goes to the winner's feature and, negated, to the leaf's.
//   k_query      : the point-query operator Q as an index: the winner leaf of
//                  the posed cell holding each point (-1 when empty / outside).
//   k_flut_adam  : Adam update of a FLUT array, then a projection onto
//                  [lower, inf) (densities stay non-negative).
#include "device_util.h"
#include "internal.h"

namespace art {

template <int ST>
__device__ inline float flut_feat(const void* feat, size_t idx) {
    if constexpr (ST == 0) return reinterpret_cast<const float*>(feat)[idx];
    else return bf16_to_f32(reinterpret_cast<const uint16_t*>(feat)[idx]);
}

// The colliding leaves of 256 consecutive leaves are listed in LDS as
// (winner, leaf) pairs; the pairs are then processed with one thread per
// (pair, channel), so the 16 (C) threads of one pair update consecutive words
// of the two FLUT rows with each atomic instruction.
template <int ST>
__global__ __launch_bounds__(256) void k_vrt(const uint32_t* __restrict__ rows, const uint32_t* __restrict__ occ_win,
                                             uint32_t n, int C, const void* __restrict__ feat,
                                             const PoseCounters* __restrict__ cnt, float lambda,
                                             float* __restrict__ d_feat, double* __restrict__ loss) {
    __shared__ double part[256 / kWave];
    __shared__ uint32_t s_win[256], s_leaf[256];
    __shared__ uint32_t s_n;
    const size_t p = blockIdx.y;
    rows += p * n;
    occ_win += p * n;
    const uint32_t nv = n - cnt[p].dropped;
    const float scale = nv ? lambda / (float)nv : 0.0f;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    double acc = 0.0;
    const int cc = (int)threadIdx.x % C, sub = (int)threadIdx.x / C, per = 256 / C;
    for (uint32_t base = blockIdx.x * 256u; base < n; base += gridDim.x * 256u) {
        const uint32_t i = base + threadIdx.x;
        uint32_t w = 0;
        bool lose = false;
        if (i < n) {
            const uint32_t row = rows[i];
            if (row != kInvalidKey) {
                w = occ_win[row];
                lose = w != i;   // a winner's Q is its own feature: no term
            }
        }
        if (lose) {
            const uint32_t k = atomicAdd(&s_n, 1u);
            s_win[k] = w;
            s_leaf[k] = i;
        }
        __syncthreads();
        const uint32_t m = s_n;
        for (uint32_t e = (uint32_t)sub; e < m; e += (uint32_t)per) {
            const uint32_t wi = s_win[e], li = s_leaf[e];
            const float diff = flut_feat<ST>(feat, (size_t)wi * C + cc) - flut_feat<ST>(feat, (size_t)li * C + cc);
            acc += (double)fabsf(diff);
            const float g = diff > 0.0f ? scale : (diff < 0.0f ? -scale : 0.0f);
            if (g != 0.0f) {
                unsafeAtomicAdd(&d_feat[(size_t)wi * C + cc], g);
                unsafeAtomicAdd(&d_feat[(size_t)li * C + cc], -g);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < 256 / kWave; ++q) t += part[q];
        if (t != 0.0) unsafeAtomicAdd(loss, t * (double)scale);
    }
}

hipError_t launch_vrt(const uint32_t* rows, const uint32_t* occ_win, uint32_t n, int C, int storage,
                      const void* feat, const PoseCounters* cnt, float lambda, int batch, float* d_feat,
                      double* loss, hipStream_t st) {
    int grid = (int)((n + 255) / 256);
    if (grid > 1024) grid = 1024;
    if (storage)
        hipLaunchKernelGGL(k_vrt<1>, dim3(grid, batch), dim3(256), 0, st, rows, occ_win, n, C, feat, cnt, lambda,
                           d_feat, loss);
    else
        hipLaunchKernelGGL(k_vrt<0>, dim3(grid, batch), dim3(256), 0, st, rows, occ_win, n, C, feat, cnt, lambda,
                           d_feat, loss);
    return hipGetLastError();
}

// Bricks are sorted by key: binary search, then the leaf's bit and its rank.
__global__ __launch_bounds__(256) void k_query(const double* __restrict__ pts, int64_t n, int depth,
                                               const uint32_t* __restrict__ brick_key,
                                               const uint32_t* __restrict__ brick_row,
                                               const uint32_t* __restrict__ brick_mask,
                                               const uint32_t* __restrict__ occ_win,
                                               const PoseCounters* __restrict__ cnt, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double invh = (double)(1 << depth);
    const int G = 2 << depth;
    int c[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = floor((pts[3 * i + a] + 1.0) * invh);
        ok = ok && u >= 0.0 && u < (double)G;
        c[a] = ok ? (int)u : 0;
    }
    int32_t res = -1;
    if (ok) {
        const uint32_t key = morton3((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]);
        const uint32_t bk = key >> 9;
        uint32_t lo = 0, hi = cnt[0].nb;   // first brick key >= bk
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (brick_key[mid] < bk) lo = mid + 1;
            else hi = mid;
        }
        if (lo < cnt[0].nb && brick_key[lo] == bk) {
            const uint32_t local = key & 511u;
            const uint32_t* m = brick_mask + (size_t)lo * 16;
            if ((m[local >> 5] >> (local & 31u)) & 1u) {
                uint32_t below = (uint32_t)__popc(m[local >> 5] & ((1u << (local & 31u)) - 1u));
                for (uint32_t j = 0; j < (local >> 5); ++j) below += (uint32_t)__popc(m[j]);
                res = (int32_t)occ_win[brick_row[lo] + below];
            }
        }
    }
    out[i] = res;
}

hipError_t launch_query(const double* pts, int64_t n, int depth, const OctreeSlot& o, const PoseCounters* cnt,
                        int32_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_query, dim3((unsigned)grid), dim3(256), 0, st, pts, n, depth, (const uint32_t*)o.brick_key,
                       (const uint32_t*)o.brick_row, (const uint32_t*)o.brick_mask, (const uint32_t*)o.occ_win, cnt,
                       out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_flut_adam(float* __restrict__ param, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t count,
                                                   AdamStep a, float lower) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float g = grad[i];
        const float mi = a.beta1 * m[i] + (1.0f - a.beta1) * g;
        const float vi = a.beta2 * v[i] + (1.0f - a.beta2) * g * g;
        m[i] = mi;
        v[i] = vi;
        const float upd = a.lr * (mi / a.bc1) / (sqrtf(vi / a.bc2) + a.eps);
        param[i] = fmaxf(param[i] - upd, lower);
    }
}

hipError_t launch_flut_adam(float* param, const float* grad, float* m, float* v, int64_t count, const AdamStep& a,
                            float lower, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t grid = (count + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_flut_adam, dim3((unsigned)grid), dim3(256), 0, st, param, grad, m, v, count, a, lower);
    return hipGetLastError();
}

}  // namespace art
