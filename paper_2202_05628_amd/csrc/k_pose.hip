// Skeleton and skinning kernels (Section 3.1, "Rigging and Deformation", Eq. 4).
//
//   k_fk   : one workgroup per pose composes the bone chain in FP64 and writes
//            the skinning matrices B_j = M^t_j (M^c_j)^-1 (FP64 and an FP32 copy).
//   k_skin : one thread per leaf blends its four bone matrices with its skin
//            weights, moves the leaf centre and writes the Morton key of the
//            posed cell (or the invalid key for a leaf outside the posed root)
//            plus its own index as the sort payload.  Leaf geometry is read as
//            SoA planes (ijk, bone ids, weights), so consecutive threads read
//            consecutive addresses of every plane.
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace art {

__device__ inline void mat3_mul(const double* A, const double* B, double* C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// G: scratch [P][J][12] (row-major 3x4 posed joint transforms).
// One workgroup per pose, one thread per bone (J <= 255 < 256 threads): the
// bones' rotations R_j (axis-angle, Rodrigues) are independent and computed
// in parallel into LDS; one thread then composes the chain in bone order
// (parent[j] < j) from LDS - only the 3x3 products and offsets are serial,
// with no global-memory round trip per bone - and the threads write G, B and
// its FP32 copy in parallel.
constexpr int kFkThreads = 256;
__global__ __launch_bounds__(kFkThreads) void k_fk(const int32_t* __restrict__ parent, const double* __restrict__ rest,
                                                   const double* __restrict__ pose, int J, int P,
                                                   double* __restrict__ G, double* __restrict__ B64,
                                                   float* __restrict__ B32) {
    __shared__ double s_R[kFkThreads][9];   // local rotation of each bone (the root's with the global one)
    __shared__ double s_G[kFkThreads][12];  // posed joint transforms
    const int p = blockIdx.x;
    const int j = threadIdx.x;
    const double* pr = pose + (size_t)p * (J + 2) * 3;
    const double* Rg = pr + (size_t)J * 3;
    const double* Tg = Rg + 3;
    if (j < J) {
        double Rj[9];
        axis_angle_to_matrix(pr + 3 * j, Rj);
        if (parent[j] < 0) {
            double Rglob[9];
            axis_angle_to_matrix(Rg, Rglob);
            mat3_mul(Rglob, Rj, s_R[j]);
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) s_R[j][e] = Rj[e];
        }
    }
    __syncthreads();
    if (j == 0) {
        for (int b = 0; b < J; ++b) {
            const double* Jb = rest + 3 * b;
            const int pa = parent[b];
            double Rot[9], t[3];
            if (pa < 0) {
#pragma unroll
                for (int e = 0; e < 9; ++e) Rot[e] = s_R[b][e];
                t[0] = Jb[0] + Tg[0];
                t[1] = Jb[1] + Tg[1];
                t[2] = Jb[2] + Tg[2];
            } else {
                const double* Gq = s_G[pa];
                const double Rq[9] = {Gq[0], Gq[1], Gq[2], Gq[4], Gq[5], Gq[6], Gq[8], Gq[9], Gq[10]};
                mat3_mul(Rq, s_R[b], Rot);
                const double* Jq = rest + 3 * pa;
                const double off[3] = {Jb[0] - Jq[0], Jb[1] - Jq[1], Jb[2] - Jq[2]};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    t[a] = Rq[3 * a] * off[0] + Rq[3 * a + 1] * off[1] + Rq[3 * a + 2] * off[2] + Gq[4 * a + 3];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s_G[b][4 * a + 0] = Rot[3 * a + 0];
                s_G[b][4 * a + 1] = Rot[3 * a + 1];
                s_G[b][4 * a + 2] = Rot[3 * a + 2];
                s_G[b][4 * a + 3] = t[a];
            }
        }
    }
    __syncthreads();
    if (j < J) {
        const double* Jj = rest + 3 * j;
        const double* Gs = s_G[j];
        double* Gj = G + ((size_t)p * J + j) * 12;
        double* Bj = B64 + ((size_t)p * J + j) * 12;
        float* Bf = B32 + ((size_t)p * J + j) * 12;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double r0 = Gs[4 * a + 0], r1 = Gs[4 * a + 1], r2 = Gs[4 * a + 2], t = Gs[4 * a + 3];
            Gj[4 * a + 0] = r0;
            Gj[4 * a + 1] = r1;
            Gj[4 * a + 2] = r2;
            Gj[4 * a + 3] = t;
            // B_j = G_j [I | -J_j]
            const double tb = t - (r0 * Jj[0] + r1 * Jj[1] + r2 * Jj[2]);
            Bj[4 * a + 0] = r0;
            Bj[4 * a + 1] = r1;
            Bj[4 * a + 2] = r2;
            Bj[4 * a + 3] = tb;
            Bf[4 * a + 0] = (float)r0;
            Bf[4 * a + 1] = (float)r1;
            Bf[4 * a + 2] = (float)r2;
            Bf[4 * a + 3] = (float)tb;
        }
    }
}

// Poses skinned by one workgroup (at most): the canonical leaf data (cell,
// bones, weights) is read once and kept in registers for all of them.
constexpr int kSkinPoses = 4;

// Batched over poses: workgroup row blockIdx.y skins poses ppb blockIdx.y ..
// + ppb - 1 (those below `batch`, ppb <= kSkinPoses); pose p reads B[p] and
// writes keys/vals + p * n.
template <typename R>
__global__ __launch_bounds__(256) void k_skin(const uint16_t* __restrict__ ijk,
                                              const uint8_t* __restrict__ bone,
                                              const float* __restrict__ w,
                                              uint32_t n, int depth,
                                              const R* __restrict__ Bpose, int J, int batch, int ppb,
                                              uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals,
                                              uint32_t* __restrict__ bmap, uint32_t bwords,
                                              PoseCounters* __restrict__ cnt) {
    extern __shared__ __align__(16) unsigned char s_dyn[];   // ppb * J * 12 bone-matrix entries
    R* sB = reinterpret_cast<R*>(s_dyn);
    const int p0 = (int)blockIdx.y * ppb;
    const int np = batch - p0 < ppb ? batch - p0 : ppb;
    __shared__ LdsOrTable<256> tab[kSkinPoses];   // brick-bitmap words touched by this workgroup, per pose
    for (int i = threadIdx.x; i < np * J * 12; i += blockDim.x) sB[i] = Bpose[(size_t)p0 * J * 12 + i];
#pragma unroll
    for (int pp = 0; pp < kSkinPoses; ++pp) tab[pp].init();
    __syncthreads();
    const R h = (R)1 / (R)(1 << depth);
    const R invh = (R)(1 << depth);
    const R G = (R)(2 << depth);
    const int lane = lane_id();
    // Each workgroup skins a contiguous range of leaves (neighbouring canonical
    // leaves land in few posed bricks).  The lanes of a wave hold consecutive
    // leaves, so the lanes still in the loop are a prefix of the wave (lane - 1
    // of an active lane is active).
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, 256, &lo, &hi);
    for (uint32_t base = lo; base < hi; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        if (i >= hi) break;
        const R x = (R)-0.5 + ((R)ijk[i] + (R)0.5) * h;
        const R y = (R)-0.5 + ((R)ijk[n + i] + (R)0.5) * h;
        const R z = (R)-0.5 + ((R)ijk[2 * (size_t)n + i] + (R)0.5) * h;
        int bk[4];
        R wk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            bk[k] = bone[(size_t)k * n + i];
            wk[k] = (R)w[(size_t)k * n + i];
        }
        for (int pp = 0; pp < np; ++pp) {
            const int p = p0 + pp;
            const R* sBp = sB + (size_t)pp * J * 12;
            R A[12];
#pragma unroll
            for (int e = 0; e < 12; ++e) A[e] = (R)0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const R* Bb = sBp + bk[k] * 12;
#pragma unroll
                for (int e = 0; e < 12; ++e) A[e] += wk[k] * Bb[e];
            }
            uint32_t c[3];
            bool ok = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R pa = A[4 * a] * x + A[4 * a + 1] * y + A[4 * a + 2] * z + A[4 * a + 3];
                const R u = floor((pa + (R)1) * invh);
                ok = ok && (u >= (R)0) && (u < G);
                c[a] = ok ? (uint32_t)u : 0u;
            }
            const uint32_t key = ok ? morton3(c[0], c[1], c[2]) : kInvalidKey;
            keys[(size_t)p * n + i] = key;
            if (vals) vals[(size_t)p * n + i] = i;
            if (bmap) {
                // mark the leaf's brick (key >> 9) in the occupancy bitmap: the bits
                // of each run of lanes with the same bitmap word are OR-ed into the
                // run's first lane, which merges them into the workgroup's table
                const uint32_t wkey = ok ? key >> 14 : kInvalidKey;
                uint32_t bits = ok ? 1u << ((key >> 9) & 31u) : 0u;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) {
                    const uint32_t ob = __shfl_down(bits, d, kWave);
                    const uint32_t ow = __shfl_down(wkey, d, kWave);
                    if (lane + d < kWave && i + (uint32_t)d < hi && ow == wkey) bits |= ob;
                }
                const uint32_t prev = __shfl_up(wkey, 1, kWave);
                if (ok && (lane == 0 || prev != wkey) && !tab[pp].insert(wkey, bits))
                    atomicOr(&bmap[(size_t)p * bwords + wkey], bits);
                const uint64_t drop = __ballot(!ok);
                if (lane == 0 && drop) atomicAdd(&cnt[p].dropped, (uint32_t)__popcll(drop));
            }
        }
    }
    if (bmap) {
        __syncthreads();
        for (int pp = 0; pp < np; ++pp)
            for (int e = threadIdx.x; e < 256; e += blockDim.x)
                if (tab[pp].key[e] != kInvalidKey) atomicOr(&bmap[(size_t)(p0 + pp) * bwords + tab[pp].key[e]], tab[pp].bits[e]);
    }
}

hipError_t launch_fk(const int32_t* parent, const double* rest, const double* pose, int J, int P,
                     double* G, double* B64, float* B32, hipStream_t st) {
    if (J < 1 || J > kFkThreads || P < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fk, dim3((unsigned)P), dim3(kFkThreads), 0, st, parent, rest, pose, J, P, G, B64, B32);
    return hipGetLastError();
}

hipError_t launch_skin(const uint16_t* ijk, const uint8_t* bone, const float* w, int64_t n,
                       int depth, const double* B64, const float* B32, int J, bool fp32, int batch,
                       uint32_t* keys, uint32_t* vals, uint32_t* bmap, uint32_t bwords, PoseCounters* cnt,
                       hipStream_t st) {
    const int bs = 256;
    int grid = (int)((n + bs - 1) / bs);
    if (grid > 1024) grid = 1024;
    // poses per workgroup: up to kSkinPoses, their bone matrices within 48 KB of LDS
    const size_t per_pose = (size_t)J * 12 * (fp32 ? 4 : 8);
    int ppb = (int)std::min<size_t>((size_t)kSkinPoses, std::max<size_t>(1, (size_t)49152 / per_pose));
    ppb = std::min(ppb, std::max(batch, 1));
    const unsigned gy = (unsigned)((batch + ppb - 1) / ppb);
    if (fp32)
        hipLaunchKernelGGL(k_skin<float>, dim3(grid, gy), dim3(bs), (size_t)ppb * per_pose, st, ijk, bone, w,
                           (uint32_t)n, depth, B32, J, batch, ppb, keys, vals, bmap, bwords, cnt);
    else
        hipLaunchKernelGGL(k_skin<double>, dim3(grid, gy), dim3(bs), (size_t)ppb * per_pose, st, ijk, bone, w,
                           (uint32_t)n, depth, B64, J, batch, ppb, keys, vals, bmap, bwords, cnt);
    return hipGetLastError();
}

}  // namespace art
