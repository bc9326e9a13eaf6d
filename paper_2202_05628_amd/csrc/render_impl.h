// Ray indexing + front-to-back compositing (Section 3.1, "Dynamic Volume
// Rendering", Eq. 5 and Eq. 6) and its adjoint.
//
// One wave64 owns one 8x8-pixel tile; a workgroup holds 2x2 tiles.  The
// tile's front-to-back brick list (see k_bin.hip) is streamed through LDS in
// chunks of 64 bricks: each lane stages one brick (its 512-bit occupancy mask,
// per-word prefix popcounts, first row and coordinates), then every lane walks
// its own ray through the staged bricks with its own cursor:
//   - a lane without a current brick slab-tests the next staged brick;
//   - a lane inside a brick takes one step of the exact ray/voxel partition:
//     the segment up to the next lattice-plane crossing, whose midpoint cell
//     is looked up in the LDS mask; an occupied cell's row in the posed FLUT
//     is brick_row + prefix + popcount(mask bits below);
//   - the sample is composited in FP32 (w = T alpha, F += w f, A += w,
//     T -= T alpha) and the lane stops once T < lambda_th.
// A wave ballot ends the chunk (and the tile) as soon as no lane has work.
// Geometry (ray parameter t, plane crossings, midpoint cells) runs in R =
// double (default) or float (precision form); compositing is always FP32.
//
// Workgroups are remapped so that each XCD (workgroups are dispatched round
// robin over the 8 XCDs) receives runs of kXcdChunk neighbouring workgroups,
// keeping neighbouring tiles - which read the same bricks and FLUT rows - in
// one XCD's L2.
#pragma once

#include "device_util.h"
#include "internal.h"

namespace art {

constexpr int kXcdChunk = 8;
constexpr int kStage = 64;

struct RArgs {
    const CamParams* cam;
    int v0, Vg, V, H, W, TX, TY, TPV, depth;
    int n_wg, wg_x, wg_per_view;
    float lambda;
    const uint32_t* tile_start;
    const uint32_t* tile_end;
    const uint32_t* pair_v;
    const uint32_t* brick_key;
    const uint32_t* brick_row;
    const uint32_t* brick_mask;
    const uint32_t* occ_win;
    const void* psig;
    const void* pfeat;
    // every per-view array below starts at the group's first view v0
    float* out_feat;      // [Vg][C][H][W]
    float* out_alpha;     // [Vg][H][W]
    float* out_tfinal;    // [Vg][H][W] or null
    const float* fwd_feat;
    const float* fwd_tfinal;
    const float* d_feat;
    const float* d_alpha;
    float* d_sigma;
    float* d_leaf_feat;
    int max_hits;
    int32_t* hit_leaf;
    double* hit_delta;
    int32_t* hit_count;
    unsigned long long* stats;   // RunStats
    const PoseCounters* counters;
};

template <int C, int ST>
__device__ inline void load_sample(const void* psig, const void* pfeat, uint32_t row, float& sg,
                                   float* f) {
    if constexpr (ST == 0) {
        sg = reinterpret_cast<const float*>(psig)[row];
        const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(pfeat) +
                                                          (size_t)row * C);
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            const float4 v = p[q];
            f[4 * q + 0] = v.x;
            f[4 * q + 1] = v.y;
            f[4 * q + 2] = v.z;
            f[4 * q + 3] = v.w;
        }
    } else {
        sg = bf16_to_f32(reinterpret_cast<const uint16_t*>(psig)[row]);
        const uint16_t* base = reinterpret_cast<const uint16_t*>(pfeat) + (size_t)row * C;
        if constexpr (C % 8 == 0) {
            const uint4* p = reinterpret_cast<const uint4*>(base);
#pragma unroll
            for (int q = 0; q < C / 8; ++q) {
                const uint4 v = p[q];
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    f[8 * q + 2 * r] = __uint_as_float(w[r] << 16);
                    f[8 * q + 2 * r + 1] = __uint_as_float(w[r] & 0xFFFF0000u);
                }
            }
        } else {
            const uint2 v = *reinterpret_cast<const uint2*>(base);
            f[0] = __uint_as_float(v.x << 16);
            f[1] = __uint_as_float(v.x & 0xFFFF0000u);
            f[2] = __uint_as_float(v.y << 16);
            f[3] = __uint_as_float(v.y & 0xFFFF0000u);
        }
    }
}

__device__ inline uint32_t spread3_small(uint32_t v) {   // 3-bit x -> bits 0, 3, 6
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4);
}

template <typename R>
__device__ inline R tplane(int k, R h, R q, R inv) {
    return ((R)k * h - q) * inv;
}

// MODE: 0 forward, 1 adjoint, 2 forward recording hit lists
template <int C, int ST, typename R, int MODE>
__global__ __launch_bounds__(256) void k_render(RArgs a) {
    __shared__ uint32_t s_mask[4][16][kStage];
    __shared__ uint16_t s_pref[4][16][kStage];
    __shared__ uint32_t s_row[4][kStage];
    __shared__ uint32_t s_coord[4][kStage];

    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;

    // XCD-aware workgroup remap
    const uint32_t hw = blockIdx.x;
    const uint32_t xcd = hw & 7u;
    const uint32_t kk = hw >> 3;
    const uint32_t wg = ((kk / kXcdChunk) * 8u + xcd) * kXcdChunk + (kk % kXcdChunk);
    if (wg >= (uint32_t)a.n_wg) return;
    // the tile lists of this group overflowed their buffer: the host re-runs it
    if (a.counters->overflow) return;

    const int vv = (int)(wg / (uint32_t)a.wg_per_view);
    const int rem = (int)(wg % (uint32_t)a.wg_per_view);
    const int ty = 2 * (rem / a.wg_x) + (wv >> 1);
    const int tx = 2 * (rem % a.wg_x) + (wv & 1);
    const bool tile_ok = tx < a.TX && ty < a.TY;
    const int px = tx * 8 + (lane & 7);
    const int py = ty * 8 + (lane >> 3);
    const bool pix_ok = tile_ok && px < a.W && py < a.H;
    const int v = a.v0 + vv;

    uint32_t ls = 0, le = 0;
    if (tile_ok) {
        const int tile = vv * a.TPV + ty * a.TX + tx;
        ls = a.tile_start[tile];
        le = a.tile_end[tile];
    }

    // ---- ray r_p = (o, d) of pixel (px, py) -----------------------------------
    const CamParams& cam = a.cam[v];
    const R h = (R)1 / (R)(1 << a.depth);
    const R invh = (R)(1 << a.depth);
    const int G = 2 << a.depth;
    R o[3], d[3], q[3], inv[3];
    {
        const R dcx = ((R)px + (R)0.5 - (R)cam.cx) / (R)cam.fx;
        const R dcy = ((R)py + (R)0.5 - (R)cam.cy) / (R)cam.fy;
        R n2 = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            d[i] = (R)cam.R[3 * i] * dcx + (R)cam.R[3 * i + 1] * dcy + (R)cam.R[3 * i + 2];
            n2 += d[i] * d[i];
        }
        const R nrm = sqrt(n2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            d[i] = d[i] / nrm;
            o[i] = (R)cam.t[i];
            q[i] = (R)1 + o[i];
            inv[i] = d[i] != (R)0 ? (R)1 / d[i] : (R)0;
        }
    }
    // clip to the posed root [-1, 1]^3 (lattice planes 0 and G)
    R ta = 0, tb = (R)INFINITY;
    bool hit_root = true;
    int c0[3];   // constant cell coordinate along axes the ray does not move on
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        c0[i] = 0;
        if (d[i] == (R)0) {
            const R u = floor(q[i] * invh);
            hit_root = hit_root && (u >= (R)0) && (u < (R)G);
            c0[i] = hit_root ? (int)u : 0;
        } else {
            const R u0 = tplane<R>(0, h, q[i], inv[i]);
            const R u1 = tplane<R>(G, h, q[i], inv[i]);
            ta = fmax(ta, fmin(u0, u1));
            tb = fmin(tb, fmax(u0, u1));
        }
    }
    bool active = pix_ok && hit_root && (tb > ta) && (ls < le);

    // ---- per-lane accumulators --------------------------------------------------
    float T = 1.0f, Aacc = 0.0f;
    float F[C];
#pragma unroll
    for (int c = 0; c < C; ++c) F[c] = 0.0f;
    int nsamp = 0;
    const size_t pix = (size_t)py * a.W + px;
    const size_t HW = (size_t)a.H * a.W;
    // adjoint state
    float g[C], Ff[C], P[C];
    float gA = 0.0f, Tfin = 0.0f;
    if constexpr (MODE == 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            g[c] = 0.0f;
            Ff[c] = 0.0f;
            P[c] = 0.0f;
        }
        if (active) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                g[c] = a.d_feat[((size_t)vv * C + c) * HW + pix];
                Ff[c] = a.fwd_feat[((size_t)vv * C + c) * HW + pix];
            }
            gA = a.d_alpha ? a.d_alpha[(size_t)vv * HW + pix] : 0.0f;
            Tfin = a.fwd_tfinal[(size_t)vv * HW + pix];
        }
    }
    const size_t hit_base = (size_t)((size_t)vv * HW + pix) * (size_t)(MODE == 2 ? a.max_hits : 0);

    // ---- traversal state --------------------------------------------------------
    bool inb = false;
    R s = 0, t1 = 0;
    R tc[3];
    int kp[3];
    int bxyz[3] = {0, 0, 0};
    int slot = 0;
    int steps = 0;

    for (uint32_t base = ls; base < le; base += kStage) {
        if (__ballot(active) == 0ull) break;
        // stage up to 64 bricks of the tile's list
        {
            const uint32_t e = base + (uint32_t)lane;
            if (e < le) {
                const uint32_t b = a.pair_v[e];
                const uint32_t bk = a.brick_key[b];
                s_coord[wv][lane] = compact3(bk) | (compact3(bk >> 1) << 10) | (compact3(bk >> 2) << 20);
                s_row[wv][lane] = a.brick_row[b];
                const uint4* mp = reinterpret_cast<const uint4*>(a.brick_mask + (size_t)b * 16);
                uint32_t run = 0;
#pragma unroll
                for (int qd = 0; qd < 4; ++qd) {
                    const uint4 m4 = mp[qd];
                    const uint32_t mw[4] = {m4.x, m4.y, m4.z, m4.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        s_mask[wv][4 * qd + r][lane] = mw[r];
                        s_pref[wv][4 * qd + r][lane] = (uint16_t)run;
                        run += (uint32_t)__popc(mw[r]);
                    }
                }
            }
        }
        wave_sync();
        const int nchunk = (int)((le - base) < (uint32_t)kStage ? (le - base) : (uint32_t)kStage);
        int cur = 0;
        while (true) {
            // a lane outside a brick slab-tests its next staged brick
            if (active && !inb && cur < nchunk) {
                const uint32_t cc = s_coord[wv][cur];
                const int b3[3] = {(int)(cc & 1023u), (int)((cc >> 10) & 1023u), (int)(cc >> 20)};
                R t0 = ta, tt1 = tb;
                bool ok = true;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (d[i] == (R)0) {
                        ok = ok && ((c0[i] >> 3) == b3[i]);
                    } else {
                        const R u0 = tplane<R>(8 * b3[i], h, q[i], inv[i]);
                        const R u1 = tplane<R>(8 * b3[i] + 8, h, q[i], inv[i]);
                        t0 = fmax(t0, fmin(u0, u1));
                        tt1 = fmin(tt1, fmax(u0, u1));
                    }
                }
                if (ok && tt1 > t0) {
                    inb = true;
                    slot = cur;
                    s = t0;
                    t1 = tt1;
                    steps = 0;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        bxyz[i] = b3[i];
                        if (d[i] == (R)0) {
                            tc[i] = (R)INFINITY;
                            kp[i] = 0;
                            continue;
                        }
                        const int lo = 8 * b3[i];
                        const R u = (q[i] + t0 * d[i]) * invh;
                        int k;
                        if (d[i] > (R)0) {
                            k = (int)floor(u) + 1;
                            k = k < lo + 1 ? lo + 1 : (k > lo + 8 ? lo + 8 : k);
                            while (k > lo + 1 && tplane<R>(k - 1, h, q[i], inv[i]) > t0) --k;
                            while (k < lo + 8 && tplane<R>(k, h, q[i], inv[i]) <= t0) ++k;
                        } else {
                            k = (int)ceil(u) - 1;
                            k = k < lo ? lo : (k > lo + 7 ? lo + 7 : k);
                            while (k < lo + 7 && tplane<R>(k + 1, h, q[i], inv[i]) > t0) ++k;
                            while (k > lo && tplane<R>(k, h, q[i], inv[i]) <= t0) --k;
                        }
                        kp[i] = k;
                        tc[i] = tplane<R>(k, h, q[i], inv[i]);
                    }
                }
                ++cur;
            }
            const bool busy = active && (inb || cur < nchunk);
            if (__ballot(busy) == 0ull) break;
            if (active && inb) {
                // one segment of the exact partition
                R s1 = fmin(fmin(tc[0], tc[1]), fmin(tc[2], t1));
                s1 = fmax(s1, s);
                if (s1 > s) {
                    const R mid = (s + s1) * (R)0.5;
                    int l[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const int c = d[i] == (R)0 ? c0[i] : (int)floor((q[i] + mid * d[i]) * invh);
                        l[i] = c - 8 * bxyz[i];
                    }
                    if ((unsigned)l[0] < 8u && (unsigned)l[1] < 8u && (unsigned)l[2] < 8u) {
                        const uint32_t m9 = spread3_small((uint32_t)l[0]) |
                                            (spread3_small((uint32_t)l[1]) << 1) |
                                            (spread3_small((uint32_t)l[2]) << 2);
                        const uint32_t wd = m9 >> 5, bit = m9 & 31u;
                        const uint32_t mw = s_mask[wv][wd][slot];
                        if ((mw >> bit) & 1u) {
                            const uint32_t row = s_row[wv][slot] + s_pref[wv][wd][slot] +
                                                 (uint32_t)__popc(mw & ((1u << bit) - 1u));
                            const float dl = (float)(s1 - s);
                            float sg;
                            float f[C];
                            load_sample<C, ST>(a.psig, a.pfeat, row, sg, f);
                            const float tau = sg * dl;
                            const float al = -expm1f(-tau);
                            const float w = T * al;
                            const float Tn = __fmaf_rn(-T, al, T);
                            if constexpr (MODE == 1) {
#pragma unroll
                                for (int c = 0; c < C; ++c) P[c] = __fmaf_rn(w, f[c], P[c]);
                                float acc = 0.0f;
#pragma unroll
                                for (int c = 0; c < C; ++c) acc += g[c] * (Tn * f[c] - (Ff[c] - P[c]));
                                const float ds = dl * (acc + gA * Tfin);
                                const uint32_t leaf = a.occ_win[row];
                                unsafeAtomicAdd(&a.d_sigma[leaf], ds);
#pragma unroll
                                for (int c = 0; c < C; ++c)
                                    unsafeAtomicAdd(&a.d_leaf_feat[(size_t)leaf * C + c], w * g[c]);
                            } else {
#pragma unroll
                                for (int c = 0; c < C; ++c) F[c] = __fmaf_rn(w, f[c], F[c]);
                                Aacc += w;
                                if constexpr (MODE == 2) {
                                    if (nsamp < a.max_hits) {
                                        a.hit_leaf[hit_base + nsamp] = (int32_t)a.occ_win[row];
                                        a.hit_delta[hit_base + nsamp] = (double)(s1 - s);
                                    }
                                }
                            }
                            T = Tn;
                            ++nsamp;
                            if (T < a.lambda) {
                                active = false;
                                inb = false;
                            }
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (tc[i] <= s1) {
                        kp[i] += d[i] > (R)0 ? 1 : -1;
                        tc[i] = tplane<R>(kp[i], h, q[i], inv[i]);
                    }
                }
                s = s1;
                if (s >= t1 || ++steps > 40) inb = false;
            }
        }
        wave_sync();
    }

    // ---- outputs -----------------------------------------------------------------
    if constexpr (MODE != 1) {
        if (pix_ok) {
#pragma unroll
            for (int c = 0; c < C; ++c) a.out_feat[((size_t)vv * C + c) * HW + pix] = F[c];
            a.out_alpha[(size_t)vv * HW + pix] = Aacc;
            if (a.out_tfinal) a.out_tfinal[(size_t)vv * HW + pix] = T;
            if constexpr (MODE == 2) a.hit_count[(size_t)vv * HW + pix] = nsamp;
        }
    }
    if (a.stats) {
        const uint64_t rays = __ballot(pix_ok);
        const uint64_t hits = __ballot(pix_ok && nsamp > 0);
        const unsigned long long ns = (unsigned long long)wave_sum((unsigned)nsamp);
        if (lane == 0 && rays) {
            atomicAdd(&a.stats[0], (unsigned long long)__popcll(rays));
            atomicAdd(&a.stats[1], ns);
            atomicAdd(&a.stats[2], (unsigned long long)__popcll(hits));
        }
    }
}

template <int C>
hipError_t launch_render_c(const RenderLaunch& r, const RArgs& a, unsigned grid, hipStream_t st);

}  // namespace art
