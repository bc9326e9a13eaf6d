// Ray indexing + front-to-back compositing (Section 3.1, "Dynamic Volume
// Rendering", Eq. 5 and Eq. 6) and its adjoint.
//
// Work distribution: k_tile_compact gathers the (pose, view, tile) items whose
// brick list is not empty with wave ballots (one atomic per wave), and
// k_background writes F = 0, A = 0, T = 1 for the pixels of the empty tiles.
// The compositing kernel then runs persistent single-wave workgroups that pull
// non-empty tiles from an atomic queue, so every resident wave has a tile with
// work in it; one wave64 renders one 8x8-pixel tile at a time.  The
// tile's front-to-back brick list (see k_bin.hip) is streamed through LDS in
// chunks of 64 bricks: each lane stages one brick (its 512-bit occupancy mask,
// per-word prefix popcounts, first row and coordinates), then every lane walks
// its own ray through the staged bricks with its own cursor:
//   - a lane without a current brick slab-tests the next staged brick;
//   - a lane inside a brick takes one step of the exact ray/voxel partition:
//     the segment up to the next lattice-plane crossing, whose midpoint cell
//     is looked up in the LDS mask; an occupied cell's index in the posed
//     octree is brick_row + prefix + popcount(mask bits below), and its
//     winner leaf id selects the FLUT row (the canonical FLUT is shared by
//     every pose, so it stays cache resident);
//   - the sample is composited in FP32 (w = T alpha, F += w f, A += w,
//     T -= T alpha) and the lane stops once T < lambda_th.
// A wave ballot ends the chunk (and the tile) as soon as no lane has work.
// Geometry (ray parameter t, plane crossings, midpoint cells) runs in R =
// double (default) or float (precision form); compositing is always FP32.
//
// Items are compacted in Morton tile order within each view, so consecutive
// queue entries - taken by waves at nearly the same time - are neighbouring
// tiles that read the same bricks and FLUT rows.
#pragma once

#include "background.h"
#include "device_util.h"
#include "internal.h"

namespace art {

constexpr int kStage = 64;
// Row pitch of the staged mask words and prefixes: with a pitch of 64 words
// every word of one brick falls into the same LDS bank, so lanes of a tile that
// look up different words of one brick serialise; one extra word per row puts
// word w of brick j into bank (w + j) mod 32.
#ifndef ART_LDS_PAD
#define ART_LDS_PAD 1
#endif
constexpr int kMaskPitch = kStage + ART_LDS_PAD;
constexpr int kPrefPitch = kStage + 2 * ART_LDS_PAD;
// Partition steps a lane may take per round while looking for its next
// occupied segment.  Bounding it keeps one lane that crosses empty cells from
// stalling the whole wave for many steps per composited sample.
#ifndef ART_STEPS_PER_ROUND
#define ART_STEPS_PER_ROUND 1
#endif

constexpr int kStepsPerRound = ART_STEPS_PER_ROUND;
// The adjoint's workloads (one pose, a few views) hold too few tiles to hide
// the memory latency of a round, so its lanes may cross several empty cells
// per round to reach their next sample.
#ifndef ART_STEPS_PER_ROUND_ADJ
#define ART_STEPS_PER_ROUND_ADJ 1
#endif

// 1: conservative FP32 slab test in the brick pre-pass (phase 1)
#ifndef ART_PHASE1_F32
#define ART_PHASE1_F32 1
#endif
// 1: fetch a sample's winner id one round before its FLUT row (three-stage
// pipeline: step -> winner id -> FLUT row -> composite)
#ifndef ART_ID_PREFETCH
#define ART_ID_PREFETCH 1
#endif
// 1: a ray leaves a brick when its cell does, and continues into the next
// listed brick without a ray/box test when its cell lies in it
// 1: an empty cell whose 2x2x2 block is empty jumps to the block's exit
#ifndef ART_SKIP_EMPTY
#define ART_SKIP_EMPTY 0
#endif
// 1: branch-free compositing step in the forward modes
#ifndef ART_BRANCHLESS
#define ART_BRANCHLESS 0
#endif
// parts of the tile work list
#ifndef ART_XCD_QUEUES
#define ART_XCD_QUEUES 1
#endif
#ifndef ART_CELL_EXIT
#define ART_CELL_EXIT 1
#endif

struct RArgs {
    const CamParams* cam;
    int Pb, V, H, W, TX, TY, TPV, depth;   // poses in this launch, views, image, tiles
    int Vg, ngroups;                       // view groups of the tile lists
    const uint32_t* items;                 // compacted non-empty tiles: pvi * TPV + ty * TX + tx
    const uint32_t* n_items;               // device count of items
    uint32_t* queue;                       // [8] next item of each part of the list (zeroed before the launch)
    uint32_t ncap;                         // per-pose capacity of the octree arrays (leaves)
    uint32_t pair_cap;                     // per (pose, group) capacity of the tile lists
    float lambda;
    const uint32_t* tile_start;            // [Pb][V][TPV], relative to the (pose, group) list
    const uint32_t* tile_end;
    const uint32_t* pair_v;                // [Pb][ngroups][pair_cap] brick ids
    const uint32_t* ovf;                   // [Pb][ngroups][2] overflow flag, pair count
    const uint32_t* brick_key;             // [Pb][ncap]
    const uint32_t* brick_row;             // [Pb][ncap + 1]
    const uint32_t* brick_mask;            // [Pb][ncap][16]
    const uint32_t* occ_win;               // [Pb][ncap]
    const void* sigma;                     // [n] canonical densities (FLUT)
    const void* feat;                      // [n][C] canonical features (FLUT)
    // maps of the launch's poses: [Pb][V][C][H][W] / [Pb][V][H][W]
    float* out_feat;
    float* out_alpha;
    float* out_tfinal;
    const float* fwd_feat;
    const float* fwd_tfinal;
    const float* d_feat;
    const float* d_alpha;
    float* d_sigma;
    float* d_leaf_feat;
    float* labels;                         // [Pb][V][H][W][2] interval labels (MODE 3)
    const float* interval;                 // [Pb][V][H][W][2] proposed intervals (MODE 4),
                                           // or [items][64][2] when interval_by_item
    int interval_by_item;
    float margin;                          // proposal margin (ray-parameter units)
    float f2_tau;                          // F2 threshold on T (< 0: off)
    int near_only;                         // MODE 4: only u_near is used (interval ends at t_b)
    float* out_depth;                      // [Pb][V][H][W] depth buffer (MODE 5)
    int sh_H;                              // MODE 6: SH coefficients per leaf (1, 4 or 9)
    int J;                                 // bones
    const uint8_t* dom_bone;               // [n] dominant bone of each canonical leaf (MODE 6)
    const float* bone_rot;                 // [Pb][J][12] bone transforms of the launch's poses (MODE 6)
    float depth_sigma;                     // MODE 5: density threshold of the depth buffer
    int adj_merge;                         // MODE 1: 0 never, 1 always, 2 with >= 2 tiles per workgroup
    // ray checkpoints (MODE 7 writes them, MODE 1 starts its segments from
    // them): before composited sample j S (j = 1 .. K) of a ray, record j - 1
    // = {entry t (double), T, P[C] = sum of w f so far}, C + 4 words per record
    float* ckpt;                           // [rays of the launch][K][C + 4]
    int32_t* ckpt_n;                       // [rays of the launch] records written
    int ckpt_K, ckpt_every;                // K records per ray, S samples per segment (0: no checkpoints)
    int bg_in_render;                      // the waves also write the background pixels (empty tiles)
    int max_hits;
    int debug_view;                        // view whose hit lists are recorded (MODE 2)
    int32_t* hit_leaf;                     // [H*W][max_hits] (single pose / view)
    double* hit_delta;
    int32_t* hit_count;
    unsigned long long* stats;             // RunStats
};

// C features of one FLUT row block starting at element `foff`.
template <int C, int ST>
__device__ inline void load_feat(const void* pfeat, size_t foff, float* f) {
    if constexpr (ST == 0) {
        const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(pfeat) + foff);
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            const float4 v = p[q];
            f[4 * q + 0] = v.x;
            f[4 * q + 1] = v.y;
            f[4 * q + 2] = v.z;
            f[4 * q + 3] = v.w;
        }
    } else {
        const uint16_t* base = reinterpret_cast<const uint16_t*>(pfeat) + foff;
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

// A FLUT feature row as loaded: C FP32 words, or C / 2 words of two BF16
// values each (channel 2k in the low half).  The BF16 row is widened to FP32
// where it is used, so a prefetched row holds half the registers and its load
// is waited for only when the sample is composited.
template <int C, int ST>
constexpr int kRowWords = ST == 0 ? C : C / 2;

template <int ST>
__device__ inline float row_at(const uint32_t* w, int c) {
    if constexpr (ST == 0) return __uint_as_float(w[c]);
    else return __uint_as_float((c & 1) ? (w[c >> 1] & 0xFFFF0000u) : (w[c >> 1] << 16));
}

// Density of FLUT row `row` (as FP32) and the raw feature words at element
// offset `foff`.
template <int C, int ST>
__device__ inline void load_sample_raw(const void* psig, const void* pfeat, uint32_t row, size_t foff, float& sg,
                                       uint32_t* w) {
    if constexpr (ST == 0) {
        sg = reinterpret_cast<const float*>(psig)[row];
        const uint4* p = reinterpret_cast<const uint4*>(reinterpret_cast<const float*>(pfeat) + foff);
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            const uint4 v = p[q];
            w[4 * q + 0] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
    } else {
        sg = bf16_to_f32(reinterpret_cast<const uint16_t*>(psig)[row]);
        const uint16_t* base = reinterpret_cast<const uint16_t*>(pfeat) + foff;
        if constexpr (C % 8 == 0) {
            const uint4* p = reinterpret_cast<const uint4*>(base);
#pragma unroll
            for (int q = 0; q < C / 8; ++q) {
                const uint4 v = p[q];
                w[4 * q + 0] = v.x;
                w[4 * q + 1] = v.y;
                w[4 * q + 2] = v.z;
                w[4 * q + 3] = v.w;
            }
        } else {
            const uint2 v = *reinterpret_cast<const uint2*>(base);
            w[0] = v.x;
            w[1] = v.y;
        }
    }
}

// Real spherical-harmonic basis of degree <= 2 (Eq. 2) at the unit direction
// (x, y, z): the orthonormal real harmonics ordered by degree l and then
// m = -l .. l, without the Condon-Shortley phase.  Entries beyond H are 0.
__device__ inline void sh_basis(int H, float x, float y, float z, float* Y) {
    const float k0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
    const float k1 = 0.4886025119029199f;    // sqrt(3 / (4 pi))
    const float k2 = 1.0925484305920792f;    // sqrt(15 / pi) / 2
    const float k3 = 0.31539156525252005f;   // sqrt(5 / pi) / 4
    const float k4 = 0.5462742152960396f;    // sqrt(15 / pi) / 4
    const bool d1 = H >= 4, d2 = H >= 9;
    Y[0] = k0;
    Y[1] = d1 ? k1 * y : 0.0f;
    Y[2] = d1 ? k1 * z : 0.0f;
    Y[3] = d1 ? k1 * x : 0.0f;
    Y[4] = d2 ? k2 * x * y : 0.0f;
    Y[5] = d2 ? k2 * y * z : 0.0f;
    Y[6] = d2 ? k3 * (3.0f * z * z - 1.0f) : 0.0f;
    Y[7] = d2 ? k2 * x * z : 0.0f;
    Y[8] = d2 ? k4 * (x * x - y * y) : 0.0f;
}

// Opacity alpha = 1 - exp(-tau) of one sample, tau >= 0.  Below tau = 1/32 a
// Taylor polynomial in Horner form (truncation below 3e-10 relative); above,
// 1 - 2^(-tau log2 e) with the hardware base-2 exponential (absolute error of
// a few 1e-8, i.e. below 2e-6 relative for alpha >= 0.03).
#ifndef ART_FAST_ALPHA
#define ART_FAST_ALPHA 1
#endif
__device__ inline float sample_alpha(float tau) {
#if ART_FAST_ALPHA
    if (tau < 0.03125f) {
        const float p = __fmaf_rn(tau, __fmaf_rn(tau, __fmaf_rn(tau, -1.0f / 120.0f, 1.0f / 24.0f), -1.0f / 6.0f), 0.5f);
        return tau * __fmaf_rn(-tau, p, 1.0f);
    }
    return 1.0f - __builtin_amdgcn_exp2f(-tau * 1.4426950408889634f);
#else
    return -expm1f(-tau);
#endif
}

__device__ inline uint32_t spread3_small(uint32_t v) {   // 3-bit x -> bits 0, 3, 6
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4);
}

// In-brick Morton index of cell (x, y, z), each in [0, 8): one byte permute
// looks the three coordinates up in the 8-entry table of spread3_small values
// (bytes 0x00 01 08 09 40 41 48 49) and two shift-or steps interleave them.
#ifndef ART_MORTON_PERM
#define ART_MORTON_PERM 1
#endif
__device__ inline uint32_t morton9_perm(uint32_t x, uint32_t y, uint32_t z) {
    const uint32_t r = __builtin_amdgcn_perm(0x49484140u, 0x09080100u, x | (y << 8) | (z << 16));
    return (r & 0xFFu) | (((r >> 8) & 0xFFu) << 1) | ((r >> 16) << 2);
}

// 1: the in-brick Morton index of a cell comes from a 512-entry LDS table
// indexed by x + 8 y + 64 z (one LDS read instead of about twenty bit
// operations per partition step; the compositing kernels are bound by their
// vector instruction issue).  Only the FP64-geometry kernels use it: the
// FP32-geometry ones run 20 single-wave workgroups per CU, whose LDS the
// table would push to the CU's limit (measured slower).
#ifndef ART_MORTON_LUT
#define ART_MORTON_LUT 1
#endif
#ifndef ART_ADJ_SORT
#define ART_ADJ_SORT 1   // 1: the adjoint merges the records of one leaf before a burst
#endif
template <typename R, int MODE>
constexpr bool kMortonLut = ART_MORTON_LUT && sizeof(R) == 8 && !(MODE == 1 && ART_ADJ_SORT);

// Ray parameter of lattice plane k on one axis: (-1 + k h - o) / d, written with
// q = 1 + o and the reciprocal of d.
template <typename R>
__device__ inline R tplane(int k, R h, R q, R inv) {
    return ((R)k * h - q) * inv;
}

// Positive-length overlap [t0, t1] of the clipped ray with brick b3.
template <typename R>
__device__ inline bool brick_overlap(const int* b3, const R* d, const R* q, const R* inv,
                                     const int* c0, R h, R ta, R tb, R& t0, R& t1) {
    t0 = ta;
    t1 = tb;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (d[i] == (R)0) {
            ok = ok && ((c0[i] >> 3) == b3[i]);
        } else {
            const R u0 = tplane<R>(8 * b3[i], h, q[i], inv[i]);
            const R u1 = tplane<R>(8 * b3[i] + 8, h, q[i], inv[i]);
            t0 = fmax(t0, fmin(u0, u1));
            t1 = fmin(t1, fmax(u0, u1));
        }
    }
    return ok && (t1 > t0);
}

// Span [ta, tb] of the ray inside the posed root (lattice planes 0 and G) along
// the axes it moves on (t >= 0).
template <typename R>
__device__ inline void root_span(const R* d, const R* q, const R* inv, R h, int G, R& ta, R& tb) {
    ta = 0;
    tb = (R)INFINITY;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (d[i] != (R)0) {
            const R u0 = tplane<R>(0, h, q[i], inv[i]);
            const R u1 = tplane<R>(G, h, q[i], inv[i]);
            ta = fmax(ta, fmin(u0, u1));
            tb = fmin(tb, fmax(u0, u1));
        }
    }
}

// MODE: 0 forward, 1 adjoint, 2 forward recording hit lists, 3 interval labels,
// 4 forward guided by proposed intervals (with full-traversal fallbacks),
// 5 forward with the depth buffer (Section 3.1, paragraph "Hybrid Rendering":
// the distance along the unit ray at which it enters the first occupied voxel
// whose density is above a threshold, searched along the whole ray: a lane
// whose compositing stops early without a depth keeps traversing, without
// compositing, until it finds one; +inf when there is none),
// 6 forward with view-dependent features (Eq. 2 in Eq. 5): the FLUT holds H
// blocks of C SH coefficients per leaf, and a sample contributes
// w sum_h k_h Y_h(d^c) at the canonical direction d^c = R^T d, R the rotation
// of the leaf's dominant bone in the tile's pose,
// 7 forward recording ray checkpoints for a segmented adjoint (RArgs::ckpt)
#ifndef ART_RENDER_WAVES_PER_EU
#define ART_RENDER_WAVES_PER_EU 3
#endif
#ifndef ART_RENDER_WAVES_PER_EU_F32
#define ART_RENDER_WAVES_PER_EU_F32 5   // FP32 geometry (the BF16 form): fewer registers, two more waves
#endif
// Adjoint gradient scatter through LDS.  Each round the lanes with a sample
// append (leaf, w, dL/dsigma, lane) to a record buffer (ballot + prefix
// count); when the buffer may not hold another round, and at the end of the
// tile, the wave adds the records' gradients with atomics in one burst: the
// density gradients one record per lane, the feature gradients w g_c with
// lanes mapped to (record, channel), so the C lanes of one atomic
// instruction that share a record update consecutive words of one leaf row
// (one cache line).  Batching matters because the vector-memory counter
// retires in order: a load issued after an atomic cannot be waited for
// without waiting for the atomic, so atomics issued every round would put
// their round trip into every round of the traversal.
#ifndef ART_ADJ_LINES
#define ART_ADJ_LINES 1
#endif
#ifndef ART_ADJ_ROUNDS
#define ART_ADJ_ROUNDS 7   // rounds of records between bursts
#endif
constexpr int kAdjRec = 64 * ART_ADJ_ROUNDS;
// Row pitch of a ray's dL/dF in LDS: 16-byte rows, offset so that the rows of
// consecutive lanes start in different banks.
template <int C>
constexpr int kAdjPitch = C + 4;
template <int C>
struct AdjLds {
    float g[64 * kAdjPitch<C>];   // dL/dF of each lane's ray
    uint32_t leaf[kAdjRec];       // records: winner leaf of a composited sample,
    float w[kAdjRec];             // its weight,
    float ds[kAdjRec];            // its density gradient
    uint8_t src[kAdjRec];         // and the lane (ray) it belongs to
#if ART_ADJ_SORT
    uint16_t ord[2][kAdjRec];   // record orders of the two counting-sort passes
    uint32_t cnt[64];           // bucket counts, then bucket starts
    uint32_t merge;             // this launch merges the records of one leaf
#endif
};

// The adjoint's LDS staging (only the adjoint kernels allocate it).
template <int C, int MODE>
__device__ inline AdjLds<C>* adj_lds() {
    if constexpr (MODE == 1) {
        __shared__ AdjLds<C> s;
        return &s;
    } else {
        return nullptr;
    }
}

#if ART_ADJ_SORT
// One stable-in-practice counting-sort pass over the n buffered records
// (wave-uniform n): takes them in the order `in` (record index order when
// null) and writes the order by bucket key(leaf) in [0, NB) to `out`.  A
// record's rank within its bucket comes from an LDS atomic on the bucket's
// count; the bucket starts are the exclusive scan of the counts across the
// wave's lanes.
template <int C, int NB, typename Key>
__device__ inline void adj_sort_pass(AdjLds<C>* s, const uint16_t* in, uint16_t* out, int n, int lane, Key key) {
    static_assert(NB <= 64, "one bucket per lane");
    if (lane < NB) s->cnt[lane] = 0u;
    wave_sync();
    uint32_t rk[kAdjRec / 64];
#pragma unroll
    for (int k = 0; k < kAdjRec / 64; ++k) {
        const int p = k * 64 + lane;
        rk[k] = 0u;
        if (p < n) rk[k] = atomicAdd(&s->cnt[key(s->leaf[in ? (int)in[p] : p])], 1u);
    }
    wave_sync();
    const uint32_t c = lane < NB ? s->cnt[lane] : 0u;
    const uint32_t start = wave_inclusive_scan(c) - c;
    wave_sync();
    if (lane < NB) s->cnt[lane] = start;
    wave_sync();
#pragma unroll
    for (int k = 0; k < kAdjRec / 64; ++k) {
        const int p = k * 64 + lane;
        if (p < n) {
            const int i = in ? (int)in[p] : p;
            out[s->cnt[key(s->leaf[i])] + rk[k]] = (uint16_t)i;
        }
    }
    wave_sync();
}
#endif

// Add the gradients of the n buffered records (wave-uniform n) and empty the
// buffer.  Every float atomic is performed at the memory side, and the
// request rate bounds the adjoint.  One atomic instruction costs one request
// per 64-byte segment its lanes touch - unless lanes hit the same word, which
// splits it into many more requests (one per lane when every word is hit
// several times).  Neighbouring rays often composite
// the same leaf in the same round, so the records are first ordered by the
// low 12 bits of their leaf (two 64-bucket passes; leaves are in Morton
// order, so the leaves of a burst share few 64-byte segments of the density
// gradient), the records of one leaf (a run) are summed, and each distinct
// leaf is added once.  A leaf whose records are not adjacent (two leaves of
// the burst 4096 apart with equal low bits) is added once per run: correct,
// only slower.  The merge lengthens each burst, so it pays only where the
// request rate binds: launches with many tiles per wave (RArgs::adj_merge).
// With fewer tiles than wave slots the kernel's time is the chain of its
// longest tile, and the records are added in buffer order.
#if ART_ADJ_SORT
template <int C>
__device__ inline int adj_flush_merged(const RArgs& a, AdjLds<C>* s_adj, int n, int lane) {
    constexpr int SPI = 64 / C;   // runs per atomic instruction
    const int cc = lane % C, sub = lane / C;
    adj_sort_pass<C, 64>(s_adj, nullptr, s_adj->ord[0], n, lane, [](uint32_t l) { return l & 63u; });
    adj_sort_pass<C, 64>(s_adj, s_adj->ord[0], s_adj->ord[1], n, lane, [](uint32_t l) { return (l >> 6) & 63u; });
    const uint16_t* ord = s_adj->ord[1];
    uint16_t* head = s_adj->ord[0];   // sorted positions where a run starts
    int nd = 0;                       // runs (wave-uniform)
    for (int p0 = 0; p0 < n; p0 += 64) {
        const int p = p0 + lane;
        const bool h = p < n && (p == 0 || s_adj->leaf[ord[p]] != s_adj->leaf[ord[p - 1]]);
        const uint64_t m = __ballot(h);
        if (h)
            head[nd + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                (uint16_t)p;
        nd += __popcll(m);
    }
    wave_sync();
    for (int r = lane; r < nd; r += 64) {
        const int b = head[r], e = r + 1 < nd ? (int)head[r + 1] : n;
        float v = 0.0f;
        for (int p = b; p < e; ++p) v += s_adj->ds[ord[p]];
        unsafeAtomicAdd(&a.d_sigma[s_adj->leaf[ord[b]]], v);
    }
    for (int r0 = 0; r0 < nd; r0 += SPI) {   // wave-uniform bound
        const int r = r0 + sub;
        if (r < nd) {
            const int b = head[r], e = r + 1 < nd ? (int)head[r + 1] : n;
            float v = 0.0f;
            for (int p = b; p < e; ++p) {
                const int i = ord[p];
                v = __fmaf_rn(s_adj->w[i], s_adj->g[(int)s_adj->src[i] * kAdjPitch<C> + cc], v);
            }
            unsafeAtomicAdd(&a.d_leaf_feat[(size_t)s_adj->leaf[ord[b]] * C + cc], v);
        }
    }
    return nd;
}
#endif

// adds: leaf-gradient additions issued (records, or runs when merged).
template <int C>
__device__ inline void adj_flush(const RArgs& a, AdjLds<C>* s_adj, int& n, int lane, uint32_t& adds) {
    wave_sync();
#if ART_ADJ_SORT
    if (__builtin_amdgcn_readfirstlane(s_adj->merge)) {
        adds += (uint32_t)adj_flush_merged<C>(a, s_adj, n, lane);
        wave_sync();   // the records are read before the buffer is reused
        n = 0;
        return;
    }
#endif
    adds += (uint32_t)n;
    // records in buffer order
    constexpr int SPI = 64 / C;   // records per atomic instruction
    const int cc = lane % C, sub = lane / C;
    for (int i = lane; i < n; i += 64) unsafeAtomicAdd(&a.d_sigma[s_adj->leaf[i]], s_adj->ds[i]);
    for (int s0 = 0; s0 < n; s0 += SPI) {   // wave-uniform bound
        const int sm = s0 + sub;
        if (sm < n)
            unsafeAtomicAdd(&a.d_leaf_feat[(size_t)s_adj->leaf[sm] * C + cc],
                            s_adj->w[sm] * s_adj->g[(int)s_adj->src[sm] * kAdjPitch<C> + cc]);
    }
    wave_sync();   // the records are read before the buffer is reused
    n = 0;
}

// Run statistics of one wave (in its workgroup's LDS, written by lane 0 only),
// added to the device counters once when the wave exits: per-tile atomics on
// the same few words would serialise.
struct WaveStats {
    unsigned long long v[14];
};

// Render one non-empty tile (item = pose-in-launch * V + view, tile index).
template <int C, int ST, typename R, int MODE>
__device__ inline void render_tile(const RArgs& a, uint32_t item, uint32_t idx, int lane, WaveStats& ws,
                                   uint32_t (*s_mask)[16][kMaskPitch],
                                   uint16_t (*s_pref)[16][kPrefPitch], uint32_t (*s_row)[kStage],
                                   const uint16_t* s_mlut,
                                   uint32_t (*s_coord)[kStage], float* s_rot, AdjLds<C>* s_adj, int seg = 0) {
    constexpr int wv = 0;
    const int pvi = (int)(item / (uint32_t)a.TPV);   // pose-in-launch * V + view
    const int tile_in_view = (int)(item % (uint32_t)a.TPV);
    const int pb = pvi / a.V;
    const int v = pvi % a.V;
    const int grp = v / a.Vg;
    const size_t slot_pg = (size_t)pb * a.ngroups + grp;
    const int ty = tile_in_view / a.TX;
    const int tx = tile_in_view % a.TX;
    const bool tile_ok = true;
    const int px = tx * 8 + (lane & 7);
    const int py = ty * 8 + (lane >> 3);
    const bool pix_ok = px < a.W && py < a.H;

    const uint32_t ls = a.tile_start[item];
    const uint32_t le = a.tile_end[item];
    const uint32_t* pair_v = a.pair_v + slot_pg * a.pair_cap;
    const uint32_t* brick_key = a.brick_key + (size_t)pb * a.ncap;
    const uint32_t* brick_row = a.brick_row + (size_t)pb * (a.ncap + 1);
    const uint32_t* brick_mask = a.brick_mask + (size_t)pb * a.ncap * 16;
    const uint32_t* occ_win = a.occ_win + (size_t)pb * a.ncap;
    const size_t es = ST == 0 ? 4 : 2;
    if constexpr (MODE == 6) {
        // rotations (row-major 3x3) of the tile pose's bone transforms, for d^c = R^T d
        const float* Bp = a.bone_rot + (size_t)pb * a.J * 12;
        for (int e = lane; e < a.J * 9; e += kWave) s_rot[e] = Bp[(e / 9) * 12 + ((e % 9) / 3) * 4 + (e % 3)];
        wave_sync();
    }


    // ---- ray r_p = (o, d) of pixel (px, py) -----------------------------------
    const CamParams& cam = a.cam[v];
    const R h = (R)1 / (R)(1 << a.depth);
    const R invh = (R)(1 << a.depth);
    const int G = 2 << a.depth;
    R d[3], q[3], inv[3];
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
            q[i] = (R)1 + (R)cam.t[i];
            inv[i] = d[i] != (R)0 ? (R)1 / d[i] : (R)0;
        }
    }
    // clip to the posed root [-1, 1]^3 (lattice planes 0 and G)
    R ta, tb;
    root_span<R>(d, q, inv, h, G, ta, tb);
    bool hit_root = true;
    int c0[3];   // constant cell coordinate along axes the ray does not move on
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        c0[i] = 0;
        if (d[i] == (R)0) {
            const R u = floor(q[i] * invh);
            hit_root = hit_root && (u >= (R)0) && (u < (R)G);
            c0[i] = hit_root ? (int)u : 0;
        }
    }
    bool active = pix_ok && hit_root && (tb > ta) && (ls < le);
    const size_t pix = (size_t)py * a.W + px;
    const size_t HW = (size_t)a.H * a.W;
    const size_t map = (size_t)pvi;   // (pose-in-launch, view) map index

    // ---- proposal (MODE 4): the first pass traverses only [ts, te] ----------------
    bool prop = false;
    if constexpr (MODE == 4) {
        if (active) {
            const float2 u = reinterpret_cast<const float2*>(a.interval)[a.interval_by_item ? (size_t)idx * 64 + lane
                                                                                            : map * HW + pix];
            if (u.x <= u.y) {   // a predicted non-empty interval (u_near <= u_far)
                const R span = tb - ta;
                const R ts = fmax(ta, ta + (R)u.x * span - (R)a.margin);
                const R te = a.near_only ? tb : fmin(tb, ta + (R)u.y * span + (R)a.margin);
                // an interval (with its margin) that covers the whole span skips
                // nothing, and a fallback could only repeat the same traversal
                if (te > ts && (ts > ta || te < tb)) {
                    ta = ts;
                    tb = te;
                    prop = true;
                }
            }
        }
    }

    // ---- adjoint segment (MODE 1 with the forward's checkpoints) -----------------
    // Segment seg of a ray covers its composited samples [seg S, (seg + 1) S)
    // - the last one the rest of the ray - from the entry t, T and P recorded
    // before sample seg S to the entry t of sample (seg + 1) S.  The partition
    // restarted at a recorded entry (a lattice crossing or a brick entry)
    // gives the same cells and chords, and from the recorded T the same
    // transmittances and stop.
    float T0 = 1.0f;
    const float* ck_P = nullptr;
    bool seg_counts = true;   // the ray-level statistics are counted once, in segment 0
    if constexpr (MODE == 1) {
        if (a.ckpt_every > 0) {
            seg_counts = seg == 0;
            if (active) {
                const size_t ray = map * HW + pix;
                const int nck = a.ckpt_n[ray];
                const float* base = a.ckpt + ray * (size_t)a.ckpt_K * (C + 4);
                if (seg > nck) {
                    active = false;
                } else {
                    if (seg < nck) tb = fmin(tb, (R)*reinterpret_cast<const double*>(base + (size_t)seg * (C + 4)));
                    if (seg > 0) {
                        const float* rec = base + (size_t)(seg - 1) * (C + 4);
                        ta = fmax(ta, (R)*reinterpret_cast<const double*>(rec));
                        T0 = rec[2];
                        ck_P = rec + 3;
                    }
                }
            }
            if (__ballot(active) == 0ull) return;   // no ray of the tile has this segment
        }
    }

    // ---- per-lane accumulators --------------------------------------------------
    float T = T0, Aacc = 0.0f;
    float F[C];
#pragma unroll
    for (int c = 0; c < C; ++c) F[c] = 0.0f;
    int nsamp = 0;
    R t_first = 0, t_last = 0;   // MODE 3: entry of the first / exit of the last sample
    float zdep = INFINITY;       // MODE 5: depth
    bool cdone = false;          // MODE 5: compositing stopped, the depth search goes on
    int adj_n = 0;          // MODE 1: records in the LDS buffer (wave-uniform)
    uint32_t adj_adds = 0;  // MODE 1: leaf-gradient additions issued (wave-uniform)
    // adjoint state.  With g = dL/dF of the ray, the density gradient of
    // sample i needs g . (T_{i+1} f_i - (F - P_i)), P_i = sum_{k<=i} w_k f_k;
    // it is kept as scalars: g . (F - P_i) = gF - gP_i with gF = g . F (from
    // the forward's map) and gP_i = sum_{k<=i} w_k (g . f_k).
    float g[C];
    float gA = 0.0f, Tfin = 0.0f, gF = 0.0f, gP = 0.0f;
    if constexpr (MODE == 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) g[c] = 0.0f;
        if (active) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                g[c] = a.d_feat[(map * C + c) * HW + pix];
                gF = __fmaf_rn(g[c], a.fwd_feat[(map * C + c) * HW + pix], gF);
            }
            gA = a.d_alpha ? a.d_alpha[map * HW + pix] : 0.0f;
            Tfin = a.fwd_tfinal[map * HW + pix];
            if (ck_P) {   // a later segment: g . P at its first sample
#pragma unroll
                for (int c = 0; c < C; ++c) gP = __fmaf_rn(g[c], ck_P[c], gP);
            }
        }
#if ART_ADJ_LINES
#pragma unroll
        for (int c = 0; c < C; ++c) s_adj->g[lane * kAdjPitch<C> + c] = g[c];
        wave_sync();
#endif
    }
    const size_t hit_base = pix * (size_t)(MODE == 2 ? a.max_hits : 0);

    // ---- traversal state (current brick) ----------------------------------------
    bool inb = false;
    R s = 0, t1 = 0;
    R tc[3] = {(R)INFINITY, (R)INFINITY, (R)INFINITY};
    // index of the next lattice plane crossed on each axis (the constant cell
    // coordinate on an axis the ray does not move along); the ray's cell at s
    // is kp - 1 on axes with d > 0 and kp otherwise
    int kp[3] = {c0[0], c0[1], c0[2]};
    int lo3[3] = {0, 0, 0};  // first lattice cell of the current brick (+1 on axes with d > 0)
    bool fresh = false;      // plane state valid (set by the first brick entry)
    int slot = 0;
    int bsteps = 0;
    uint32_t row_base = 0;

    uint32_t rounds = 0;   // wave-uniform traversal rounds (diagnostic)
    uint32_t nsteps = 0;   // partition steps of this lane (diagnostic)
    uint32_t nfall = 0;    // MODE 4: this lane fell back to the full traversal
    for (int pass = 0; pass < (MODE == 4 ? 2 : 1); ++pass) {
    if constexpr (MODE == 4) {
        if (pass == 1) {
            // F1: the proposed interval held no occupied voxel; F2: the ray left
            // it with transmittance above the threshold before the root's exit.
            // Such lanes restart from t_a.
            // the whole span is recomputed rather than kept in registers
            R ta_full, tb_full;
            root_span<R>(d, q, inv, h, G, ta_full, tb_full);
            const bool fb = prop && (nsamp == 0 || (a.f2_tau >= 0.0f && T >= a.f2_tau && tb < tb_full));
            if (__ballot(fb) == 0ull) break;
            active = fb;
            if (fb) {
                // With the interval ending at t_b (near end only), F1 means that
                // [t_s, t_b] held no occupied voxel - the cell holding t_s
                // included, since a sub-chord of a cell has its midpoint in that
                // cell - so every sample of the full traversal lies in
                // [t_a, t_s): only that part is traversed again.
                const bool front_only = a.near_only && nsamp == 0;
                T = 1.0f;
                Aacc = 0.0f;
#pragma unroll
                for (int c = 0; c < C; ++c) F[c] = 0.0f;
                nsamp = 0;
                tb = front_only ? ta : tb_full;
                ta = ta_full;
                nfall = 1;
            }
            inb = false;
            fresh = false;
        }
    }
    for (uint32_t base = ls; base < le; base += kStage) {
        if (__ballot(active) == 0ull) break;
        // stage up to 64 bricks of the tile's front-to-back list
        {
            const uint32_t e = base + (uint32_t)lane;
            if (e < le) {
                const uint32_t b = pair_v[e];
                const uint32_t bk = brick_key[b];
                s_coord[wv][lane] = compact3(bk) | (compact3(bk >> 1) << 10) | (compact3(bk >> 2) << 20);
                s_row[wv][lane] = brick_row[b];
                const uint4* mp = reinterpret_cast<const uint4*>(brick_mask + (size_t)b * 16);
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
#if ART_PHASE1_F32
        // phase 1: which staged bricks may this lane's ray cross?  A
        // conservative FP32 slab test against each brick grown by kGrow on
        // every face: it never misses a brick the exact test accepts (the
        // coefficients' rounding stays far below kGrow / |d|), and phase 2
        // re-tests every brick exactly before entering it.
        uint64_t todo = 0;
        if (active) {
            constexpr double kGrow = 1e-5;
            float a8[3], a0[3], aw[3];
            bool par[3];
            // recomputed per chunk (opaque to loop-invariant hoisting) so that
            // the coefficients are not held in registers across the tile
            double hh = (double)h;
            asm volatile("" : "+v"(hh));
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                par[i] = d[i] == (R)0;
                const double iv = par[i] ? 0.0 : (double)inv[i];
                a8[i] = (float)(8.0 * hh * iv);
                a0[i] = (float)(-((double)q[i] + kGrow) * iv);
                aw[i] = (float)((8.0 * hh + 2.0 * kGrow) * iv);
            }
            const float taf = (float)ta - 1e-5f, tbf = (float)tb + 1e-5f;
#pragma unroll 1
            for (int j = 0; j < nchunk; ++j) {
                const uint32_t cc = s_coord[wv][j];
                const int b3[3] = {(int)(cc & 1023u), (int)((cc >> 10) & 1023u), (int)(cc >> 20)};
                float t0 = taf, t1f = tbf;
                bool ok = true;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (par[i]) {
                        ok = ok && ((c0[i] >> 3) == b3[i]);
                    } else {
                        const float u0 = __fmaf_rn((float)b3[i], a8[i], a0[i]);
                        const float u1 = u0 + aw[i];
                        t0 = fmaxf(t0, fminf(u0, u1));
                        t1f = fminf(t1f, fmaxf(u0, u1));
                    }
                }
                if (ok && t1f > t0) todo |= 1ull << j;
            }
        }
#else
        // phase 1: which staged bricks does this lane's ray cross (positive length)?
        uint64_t todo = 0;
        if (active) {
            for (int j = 0; j < nchunk; ++j) {
                const uint32_t cc = s_coord[wv][j];
                const int b3[3] = {(int)(cc & 1023u), (int)((cc >> 10) & 1023u), (int)(cc >> 20)};
                R u0, u1;
                if (brick_overlap<R>(b3, d, q, inv, c0, h, ta, tb, u0, u1)) todo |= 1ull << j;
            }
        }
#endif
        // phase 2: walk the crossed bricks in list order.  Software pipeline of
        // depth one: each round advances the ray to its next occupied segment
        // while the current sample's gather is in flight, composites the current
        // sample, then issues the next sample's gather into the same registers.
        bool hasA = false;
        uint32_t rowA = 0, winA = 0;
        float dlA = 0.0f;
        double dxA = 0.0;
        R sA0 = 0, sA1 = 0;
        float sgA = 0.0f;
        bool hasI = false;   // a sample whose winner id is in flight (ART_ID_PREFETCH)
        uint32_t winI = 0;
        float dlI = 0.0f;
        double dxI = 0.0;
        R sI0 = 0, sI1 = 0;
        uint32_t fA[kRowWords<C, ST>];   // the sample's feature row as loaded
#pragma unroll
        for (int c = 0; c < kRowWords<C, ST>; ++c) fA[c] = 0u;
        uint32_t domA = 0;   // MODE 6: dominant bone of the sample's leaf
        bool adj_has = false;   // MODE 1: this lane composited a sample this round
        uint32_t adj_leaf = 0;
        float adj_w = 0.0f, adj_ds = 0.0f;
        while (true) {
            const bool more = active && (inb || todo != 0ull);
            if (__ballot(more || hasA || hasI) == 0ull) break;
            ++rounds;
            // (1) next occupied segment of this lane's ray (overlaps the gather of A)
            bool hasB = false;
            uint32_t rowB = 0;
            float dlB = 0.0f;
            double dxB = 0.0;
            R sB0 = 0, sB1 = 0;
            int guard = 0;
            while (active && !hasB && (inb || todo != 0ull) &&
                   guard < (MODE == 1 ? ART_STEPS_PER_ROUND_ADJ : kStepsPerRound)) {
                ++guard;
                ++nsteps;
                if (!inb) {
                    slot = __ffsll((unsigned long long)todo) - 1;
                    todo &= todo - 1ull;
                    const uint32_t cc = s_coord[wv][slot];
                    const int b3[3] = {(int)(cc & 1023u), (int)((cc >> 10) & 1023u), (int)(cc >> 20)};
#if ART_CELL_EXIT
                    // The ray continues into this brick when its current cell (it
                    // just left the previous brick through a face) lies in it: the
                    // plane state carries over and no ray/box test is needed.
                    bool cont = fresh;
#pragma unroll
                    for (int i = 0; i < 3; ++i) cont = cont && (((kp[i] - (d[i] > (R)0 ? 1 : 0)) >> 3) == b3[i]);
                    if (!cont) {
                        R t0, t1x;
                        if (!brick_overlap<R>(b3, d, q, inv, c0, h, ta, tb, t0, t1x)) continue;
                        // restart the plane state from the lattice coordinate at t0;
                        // rounding there can only misplace a segment shorter than the
                        // rounding itself (a plane index one too small costs one
                        // empty step)
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            if (d[i] == (R)0) continue;
                            const R u = (q[i] + t0 * d[i]) * invh;
                            const int k = d[i] > (R)0 ? (int)floor(u) + 1 : (int)ceil(u) - 1;
                            kp[i] = k;
                            tc[i] = tplane<R>(k, h, q[i], inv[i]);
                        }
                        fresh = true;
                        s = t0;
                    }
                    inb = true;
                    bsteps = 0;
                    row_base = s_row[wv][slot];
#pragma unroll
                    for (int i = 0; i < 3; ++i) lo3[i] = 8 * b3[i] + (d[i] > (R)0 ? 1 : 0);
#else
                    R t0;
                    if (!brick_overlap<R>(b3, d, q, inv, c0, h, ta, tb, t0, t1)) continue;
                    inb = true;
                    bsteps = 0;
                    row_base = s_row[wv][slot];
#pragma unroll
                    for (int i = 0; i < 3; ++i) lo3[i] = 8 * b3[i] + (d[i] > (R)0 ? 1 : 0);
                    // Entering exactly where the ray left the previous brick (its
                    // neighbour), the plane state carries over unchanged.  Otherwise
                    // it restarts from the lattice coordinate at t0; rounding there
                    // can only misplace a segment shorter than the rounding itself
                    // (a plane index one too small costs one empty step).
                    if (!(fresh && t0 == s)) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            if (d[i] == (R)0) continue;
                            const R u = (q[i] + t0 * d[i]) * invh;
                            const int k = d[i] > (R)0 ? (int)floor(u) + 1 : (int)ceil(u) - 1;
                            kp[i] = k;
                            tc[i] = tplane<R>(k, h, q[i], inv[i]);
                        }
                        fresh = true;
                    }
                    s = t0;
#endif
                }
                // one segment of the exact partition: (s, s1) in the ray's cell
#if ART_CELL_EXIT
                R s1 = fmin(fmin(tc[0], tc[1]), fmin(tc[2], tb));
#else
                R s1 = fmin(fmin(tc[0], tc[1]), fmin(tc[2], t1));
#endif
                s1 = fmax(s1, s);
                const int l0 = kp[0] - lo3[0], l1 = kp[1] - lo3[1], l2 = kp[2] - lo3[2];
                if (s1 > s && (unsigned)l0 < 8u && (unsigned)l1 < 8u && (unsigned)l2 < 8u) {
                    uint32_t m9;
                    if constexpr (kMortonLut<R, MODE>)
                        m9 = s_mlut[l0 + 8 * l1 + 64 * l2];
                    else
                        m9 = ART_MORTON_PERM ? morton9_perm((uint32_t)l0, (uint32_t)l1, (uint32_t)l2)
                                             : spread3_small((uint32_t)l0) | (spread3_small((uint32_t)l1) << 1) |
                                                   (spread3_small((uint32_t)l2) << 2);
                    const uint32_t wd = m9 >> 5, bit = m9 & 31u;
                    const uint32_t mw = s_mask[wv][wd][slot];
                    if ((mw >> bit) & 1u) {
                        rowB = row_base + s_pref[wv][wd][slot] + (uint32_t)__popc(mw & ((1u << bit) - 1u));
                        dlB = (float)(s1 - s);
                        if constexpr (MODE == 2) dxB = (double)(s1 - s);
                        if constexpr (MODE == 3) {
                            sB0 = s;
                            sB1 = s1;
                        }
                        if constexpr (MODE == 5 || MODE == 7) sB0 = s;
                        hasB = true;
                    }
#if ART_SKIP_EMPTY
                    else if (((mw >> (bit & ~7u)) & 0xFFu) == 0u) {
                        // The cell's whole 2x2x2 block (8 consecutive mask bits in
                        // Morton order) is empty: jump to the block's exit face.  The
                        // exit is a lattice plane crossing computed by the same formula
                        // as the cell-by-cell steps, so the partition after the jump
                        // is unchanged; only empty segments are skipped.
                        const int lc[3] = {l0, l1, l2};
                        R tx = tb;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            if (d[i] == (R)0) continue;
                            const int pos = d[i] > (R)0 ? 1 : 0;
                            const int ke = lo3[i] - pos + (lc[i] & ~1) + 2 * pos;
                            tx = fmin(tx, tplane<R>(ke, h, q[i], inv[i]));
                        }
                        s1 = fmax(tx, s1);
                    }
#endif
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
#pragma unroll
                    for (int rep = 0; rep < (ART_SKIP_EMPTY ? 2 : 1); ++rep) {
                        if (tc[i] <= s1) {
                            const int st = d[i] > (R)0 ? 1 : -1;
                            kp[i] += st;
                            tc[i] = tplane<R>(kp[i], h, q[i], inv[i]);
                        }
                    }
                }
                s = s1;
                // a brick holds at most 3 * 8 plane crossings; the cap only guards
                // against non-finite input
#if ART_CELL_EXIT
                {   // the ray leaves the brick when its cell does
                    const int m0 = kp[0] - lo3[0], m1 = kp[1] - lo3[1], m2 = kp[2] - lo3[2];
                    const bool inside = (unsigned)m0 < 8u && (unsigned)m1 < 8u && (unsigned)m2 < 8u;
                    if (!inside || s >= tb || ++bsteps > 32) inb = false;
                }
#else
                if (s >= t1 || ++bsteps > 32) inb = false;
#endif
            }
            // (2) composite the current sample (Eq. 5-6, exclusive transmittance)
            if (MODE == 5 && cdone) {
                // depth search past the early stop: no compositing
                if (hasA && active && sgA > a.depth_sigma) {
                    zdep = (float)sA0;
                    active = false;
                    inb = false;
                }
            } else
#if ART_BRANCHLESS
            // forward without hit lists: every lane runs the update, a lane without
            // a sample with alpha = 0 (w = 0 leaves F, A and T unchanged exactly)
            if constexpr (MODE == 0 || MODE == 4) {
                const bool doA = hasA && active;
                const float al = sample_alpha(doA ? sgA * dlA : 0.0f);
                const float w = T * al;
#pragma unroll
                for (int c = 0; c < C; ++c) F[c] = __fmaf_rn(w, row_at<ST>(fA, c), F[c]);
                Aacc += w;
                T = __fmaf_rn(-T, al, T);
                nsamp += doA ? 1 : 0;
                if (doA && T < a.lambda) {
                    active = false;
                    inb = false;
                }
            } else
#endif
            if (hasA && active) {
                // no FMA contraction here: every mode rounds w = T alpha and
                // A += w identically (the FMAs below are explicit)
#pragma clang fp contract(off)
                const float tau = sgA * dlA;
                const float al = sample_alpha(tau);
                const float w = T * al;
                const float Tn = __fmaf_rn(-T, al, T);
                if constexpr (MODE == 1) {
                    float gf = 0.0f;   // g . f_i (g read back from LDS: fewer live registers)
#if ART_ADJ_LINES
                    const float4* g4 = reinterpret_cast<const float4*>(&s_adj->g[lane * kAdjPitch<C>]);
#pragma unroll
                    for (int q = 0; q < C / 4; ++q) {
                        const float4 gv = g4[q];
                        gf = __fmaf_rn(gv.x, row_at<ST>(fA, 4 * q + 0), gf);
                        gf = __fmaf_rn(gv.y, row_at<ST>(fA, 4 * q + 1), gf);
                        gf = __fmaf_rn(gv.z, row_at<ST>(fA, 4 * q + 2), gf);
                        gf = __fmaf_rn(gv.w, row_at<ST>(fA, 4 * q + 3), gf);
                    }
#else
#pragma unroll
                    for (int c = 0; c < C; ++c) gf = __fmaf_rn(g[c], row_at<ST>(fA, c), gf);
#endif
                    gP = __fmaf_rn(w, gf, gP);
                    const float acc = Tn * gf - (gF - gP);
                    const float ds = dlA * (acc + gA * Tfin);
                    const uint32_t leaf = winA;
#if ART_ADJ_LINES
                    adj_leaf = leaf;
                    adj_w = w;
                    adj_ds = ds;
                    adj_has = true;
#else
                    unsafeAtomicAdd(&a.d_sigma[leaf], ds);
#pragma unroll
                    for (int c = 0; c < C; ++c) unsafeAtomicAdd(&a.d_leaf_feat[(size_t)leaf * C + c], w * g[c]);
#endif
                } else {
                    if constexpr (MODE == 7) {
                        // checkpoint before composited sample j S (j = 1 .. K): its entry
                        // distance, T and the feature sum before it
                        const int j = nsamp / a.ckpt_every;
                        if (nsamp > 0 && nsamp == j * a.ckpt_every && j <= a.ckpt_K) {
                            float* rec = a.ckpt + ((map * HW + pix) * (size_t)a.ckpt_K + (size_t)(j - 1)) * (C + 4);
                            *reinterpret_cast<double*>(rec) = (double)sA0;
                            rec[2] = T;
#pragma unroll
                            for (int c = 0; c < C; ++c) rec[3 + c] = F[c];
                        }
                    }
                    if constexpr (MODE == 6) {
                        // S_c = sum_h k_{h,c} Y_h(R^T d); the first block is the prefetched row
                        const float* Rm = s_rot + domA * 9;
                        const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
                        float Y[9];
                        sh_basis(a.sh_H, Rm[0] * dx + Rm[3] * dy + Rm[6] * dz, Rm[1] * dx + Rm[4] * dy + Rm[7] * dz,
                                 Rm[2] * dx + Rm[5] * dy + Rm[8] * dz, Y);
                        const float w0 = w * Y[0];
#pragma unroll
                        for (int c = 0; c < C; ++c) F[c] = __fmaf_rn(w0, row_at<ST>(fA, c), F[c]);
#pragma unroll
                        for (int hb = 1; hb < 9; ++hb) {
                            if (hb < a.sh_H) {
                                float fb[C];
                                load_feat<C, ST>(a.feat, ((size_t)winA * a.sh_H + hb) * C, fb);
                                const float wy = w * Y[hb];
#pragma unroll
                                for (int c = 0; c < C; ++c) F[c] = __fmaf_rn(wy, fb[c], F[c]);
                            }
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < C; ++c) F[c] = __fmaf_rn(w, row_at<ST>(fA, c), F[c]);
                    }
                    Aacc += w;
                    if constexpr (MODE == 2) {
                        if (nsamp < a.max_hits) {
                            a.hit_leaf[hit_base + nsamp] = (int32_t)winA;
                            a.hit_delta[hit_base + nsamp] = dxA;
                        }
                    }
                    if constexpr (MODE == 3) {
                        if (nsamp == 0) t_first = sA0;
                        t_last = sA1;
                    }
                    if constexpr (MODE == 5) {
                        if (zdep == INFINITY && sgA > a.depth_sigma) zdep = (float)sA0;
                    }
                }
                T = Tn;
                ++nsamp;
                if (T < a.lambda) {
                    if (MODE == 5 && zdep == INFINITY) {
                        cdone = true;
                    } else {
                        active = false;
                        inb = false;
                    }
                }
            }
#if ART_ADJ_LINES
            if constexpr (MODE == 1) {
                const uint64_t staged = __ballot(adj_has);
                if (staged) {
                    if (adj_has) {   // append this round's samples to the records
                        const int slotc = adj_n + (int)__builtin_amdgcn_mbcnt_hi(
                                                     (uint32_t)(staged >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)staged, 0u));
                        s_adj->leaf[slotc] = adj_leaf;
                        s_adj->w[slotc] = adj_w;
                        s_adj->ds[slotc] = adj_ds;
                        s_adj->src[slotc] = (uint8_t)lane;
                    }
                    adj_n += __popcll(staged);
                    adj_has = false;
                    if (adj_n > kAdjRec - 64) adj_flush<C>(a, s_adj, adj_n, lane, adj_adds);
                }
            }
#endif
#if ART_ID_PREFETCH
            // (3) the sample whose winner id has arrived issues its FLUT gather,
            // (4) the new sample fetches its collision winner's id.  Both loads
            // are issued by every lane every round (a lane without a sample
            // reads row 0), so the wait before compositing only has to cover the
            // FLUT row and leaves the winner-id load in flight.
            hasA = hasI && active;
            dlA = dlI;
            dxA = dxI;
            sA0 = sI0;
            sA1 = sI1;
            winA = hasA ? winI : 0u;
            load_sample_raw<C, ST>(a.sigma, a.feat, winA,
                                   (size_t)winA * (MODE == 6 ? (size_t)a.sh_H * C : (size_t)C), sgA, fA);
            if constexpr (MODE == 6) domA = a.dom_bone[winA];
            hasI = hasB && active;
            dlI = dlB;
            dxI = dxB;
            sI0 = sB0;
            sI1 = sB1;
            winI = occ_win[hasI ? rowB : 0u];
#else
            // (3) issue the next sample's gather into the freed registers
            hasA = hasB && active;
            if (hasA) {
                rowA = rowB;
                dlA = dlB;
                dxA = dxB;
                sA0 = sB0;
                sA1 = sB1;
                // the FLUT row of the cell's collision winner
                winA = occ_win[rowA];
                load_sample_raw<C, ST>(a.sigma, a.feat, winA,
                                       (size_t)winA * (MODE == 6 ? (size_t)a.sh_H * C : (size_t)C), sgA, fA);
            if constexpr (MODE == 6) domA = a.dom_bone[winA];
            }
#endif
        }
        wave_sync();
    }
    }   // passes

#if ART_ADJ_LINES
    if constexpr (MODE == 1) {
        if (adj_n > 0) adj_flush<C>(a, s_adj, adj_n, lane, adj_adds);
    }
#endif

    // ---- outputs -----------------------------------------------------------------
    if constexpr (MODE == 3) {
        if (pix_ok) {
            float2 lab = make_float2(1.0f, 0.0f);   // no composited sample: empty interval
            if (nsamp > 0) {
                const R span = tb - ta;
                lab.x = (float)((t_first - ta) / span);
                lab.y = (float)((t_last - ta) / span);
            }
            reinterpret_cast<float2*>(a.labels)[map * HW + pix] = lab;
        }
    } else if constexpr (MODE != 1) {
        if (pix_ok) {
#pragma unroll
            for (int c = 0; c < C; ++c) store_stream(&a.out_feat[(map * C + c) * HW + pix], F[c]);
            store_stream(&a.out_alpha[map * HW + pix], Aacc);
            if (a.out_tfinal) store_stream(&a.out_tfinal[map * HW + pix], T);
            if constexpr (MODE == 2) a.hit_count[pix] = nsamp;
            if constexpr (MODE == 5) a.out_depth[map * HW + pix] = zdep;
            if constexpr (MODE == 7) {
                const int nck = nsamp > 0 ? (nsamp - 1) / a.ckpt_every : 0;
                a.ckpt_n[map * HW + pix] = nck < a.ckpt_K ? nck : a.ckpt_K;
            }
        }
    }
    if (a.stats) {
        const uint64_t rays = __ballot(pix_ok);
        const uint64_t hits = __ballot(pix_ok && nsamp > 0);
        const unsigned long long ns = (unsigned long long)wave_sum((unsigned)nsamp);
        const unsigned long long steps = (unsigned long long)wave_sum(nsteps);
        if (lane == 0 && rays) {   // wave-uniform values
            if (seg_counts) {
                ws.v[0] += (unsigned long long)__popcll(rays);
                ws.v[2] += (unsigned long long)__popcll(hits);
                ws.v[7] += (unsigned long long)(le - ls);
                ws.v[10] += (unsigned long long)__popcll(rays);
            }
            ws.v[1] += ns;
            ws.v[8] += (unsigned long long)rounds;
            ws.v[9] += steps;
        }
        if constexpr (MODE == 1) {
            if (lane == 0) ws.v[13] += (unsigned long long)adj_adds;
        }
        if constexpr (MODE == 4) {
            const uint64_t pr = __ballot(prop);
            const uint64_t fl = __ballot(nfall != 0u);
            if (lane == 0) {
                ws.v[11] += (unsigned long long)__popcll(pr);
                ws.v[12] += (unsigned long long)__popcll(fl);
            }
        }
    }
}

// One background chunk (kBgChunkGroups 4-pixel groups) taken from its queue
// by a wave; false when every chunk has been taken.  The chunk's geometry
// comes from the kernel arguments at each call (nothing of it stays live
// across the tiles).  Launches with background work hold fewer than 2^31
// groups (the host checks), so the 32-bit group index of a chunk cannot wrap.
template <int C>
__device__ inline bool bg_take(const RArgs& a, uint32_t n_bg, uint32_t groups, int lane, WaveStats& ws) {
    if (n_bg == 0u) return false;
    uint32_t c = 0;
    if (lane == 0) c = atomicAdd(&a.queue[8], 1u);
    c = (uint32_t)__shfl((int)c, 0, kWave);
    if (c >= n_bg) return false;
    BgArgs bg;
    bg.V = a.V;
    bg.Vg = a.Vg;
    bg.ngroups = a.ngroups;
    bg.H = a.H;
    bg.W = a.W;
    bg.C = C;
    bg.TX = a.TX;
    bg.TPV = a.TPV;
    bg.debug_view = -1;
    bg.ovf = a.ovf;
    bg.tile_start = a.tile_start;
    bg.tile_end = a.tile_end;
    bg.out_feat = a.out_feat;
    bg.out_alpha = a.out_alpha;
    bg.out_tfinal = a.out_tfinal;
    bg.labels = nullptr;
    bg.out_depth = a.out_depth;
    bg.hit_count = nullptr;
    const uint32_t HW4 = (uint32_t)a.H * (uint32_t)a.W / 4u;
    int n = 0;
#pragma unroll 1
    for (uint32_t k = 0; k < kBgChunkGroups / kWave; ++k) {
        const uint32_t i = c * kBgChunkGroups + k * kWave + (uint32_t)lane;
        if (i < groups) n += bg_group4(bg, i / HW4, i % HW4);
    }
    const unsigned long long w = (unsigned long long)wave_sum((unsigned)n);
    if (lane == 0) ws.v[0] += w;
    return true;
}

// Consecutive work-list tiles a wave takes per queue atomic.
#ifndef ART_TILES_PER_GRAB
#define ART_TILES_PER_GRAB 1
#endif

// Persistent compositing kernel: each single-wave workgroup takes non-empty
// tiles from the queue until it is exhausted (every wave reaches the exit).
template <int C, int ST, typename R, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(
    MODE == 1 ? 1 : (MODE == 6 ? 2 : (sizeof(R) == 4 ? ART_RENDER_WAVES_PER_EU_F32 : ART_RENDER_WAVES_PER_EU)))))
void k_render(RArgs a) {
    __shared__ uint32_t s_mask[1][16][kMaskPitch];
    __shared__ uint16_t s_pref[1][16][kPrefPitch];
    __shared__ uint32_t s_row[1][kStage];
    __shared__ uint32_t s_coord[1][kStage];
    __shared__ float s_rot[MODE == 6 ? kMaxBonesSH * 9 : 1];
    __shared__ uint16_t s_mlut[kMortonLut<R, MODE> ? 512 : 1];
    AdjLds<C>* s_adj = adj_lds<C, MODE>();
    const int lane = threadIdx.x & 63;
    // invalid densities in the FLUT: nothing is rendered (the call reports it)
    if (a.stats[kStatBadSigma] != 0ull) return;
    if constexpr (kMortonLut<R, MODE>) {
        for (int e = lane; e < 512; e += kWave)
            s_mlut[e] = (uint16_t)(spread3_small((uint32_t)e & 7u) | (spread3_small(((uint32_t)e >> 3) & 7u) << 1) |
                                   (spread3_small((uint32_t)e >> 6) << 2));
        wave_sync();
    }
    const uint32_t n_tiles = *a.n_items;
    // MODE 1 with checkpoints: K + 1 segments per tile, item v = (tile v / (K + 1),
    // segment v mod (K + 1)) - the segments of one tile are taken together
    const uint32_t nseg = (MODE == 1 && a.ckpt_every > 0) ? (uint32_t)a.ckpt_K + 1u : 1u;
    const uint32_t n_items = n_tiles * nseg;
#if ART_ADJ_SORT
    if constexpr (MODE == 1) {
        if (lane == 0)
            s_adj->merge = a.adj_merge == 1 || (a.adj_merge == 2 && (uint64_t)n_items >= 2ull * gridDim.x);
        wave_sync();
    }
#endif
    __shared__ WaveStats ws;
    if (lane == 0)
        for (int i = 0; i < 14; ++i) ws.v[i] = 0ull;
    // Background pixels (when this launch writes them): a wave takes a chunk
    // after every `every` tiles - spread so that the stores overlap the
    // compositing - and the remaining chunks once the work list is drained.
    uint32_t n_bg = 0, every = 0xFFFFFFFFu, since = 0, bg_groups = 0;
    if constexpr (MODE == 0 || MODE == 4 || MODE == 5 || MODE == 6 || MODE == 7) {
        if (a.bg_in_render) {
            bg_groups = (uint32_t)((uint64_t)a.Pb * a.V * a.H * a.W / 4);
            n_bg = (bg_groups + kBgChunkGroups - 1) / kBgChunkGroups;
            every = n_items / n_bg > 1u ? n_items / n_bg : 1u;
        }
    }
    // The work list may be cut into kQueues contiguous parts (neighbouring
    // tiles, which read the same bricks and FLUT rows, stay in one part);
    // workgroups are dispatched to the XCDs in turn, so a workgroup starts on
    // part blockIdx.x mod kQueues - the waves of one XCD then share its L2 -
    // and helps the other parts once its own is drained.  (One part per XCD
    // raised the L2 hit rate from 55 % to 58 % but the kernel ran 4 % longer,
    // so the default is a single queue.)
    constexpr uint32_t kQueues = ART_XCD_QUEUES;
    const uint32_t home = blockIdx.x % kQueues;
    uint32_t part = 0;
    bool tiles_left = true;
    while (true) {
        if (tiles_left) {
            const uint32_t qi = (home + part) % kQueues;
            const uint32_t beg = (uint32_t)((uint64_t)n_items * qi / kQueues);
            const uint32_t end = (uint32_t)((uint64_t)n_items * (qi + 1) / kQueues);
            uint32_t idx = 0;
            if (lane == 0) idx = atomicAdd(&a.queue[qi], (uint32_t)ART_TILES_PER_GRAB);
            idx = beg + (uint32_t)__shfl((int)idx, 0, kWave);
            if (idx >= end) {
                if (++part == kQueues) tiles_left = false;
                continue;   // the next part, or the remaining background
            }
            for (uint32_t t = 0; t < (uint32_t)ART_TILES_PER_GRAB && idx + t < end; ++t) {
                const uint32_t v = idx + t;
                render_tile<C, ST, R, MODE>(a, a.items[v / nseg], v / nseg, lane, ws, s_mask, s_pref, s_row, s_mlut,
                                            s_coord, s_rot, s_adj, (int)(v % nseg));
                wave_sync();
            }
            if (++since < every) continue;   // (every is 2^32 - 1 without background work)
            since = 0;
        }
        if (!bg_take<C>(a, n_bg, bg_groups, lane, ws) && !tiles_left) break;
    }
    if (a.stats && lane == 0)
        for (int i = 0; i < 14; ++i)
            if (ws.v[i]) atomicAdd(&a.stats[i], ws.v[i]);
}

template <int C>
hipError_t launch_render_c(const RenderLaunch& r, const RArgs& a, unsigned grid, hipStream_t st);

template <int C, int ST, typename R>
hipError_t launch_render_mode(const RenderLaunch& r, const RArgs& a, unsigned grid, hipStream_t st) {
    switch (r.mode) {
        case 0: hipLaunchKernelGGL((k_render<C, ST, R, 0>), dim3(grid), dim3(64), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_render<C, ST, R, 1>), dim3(grid), dim3(64), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_render<C, ST, R, 2>), dim3(grid), dim3(64), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_render<C, ST, R, 3>), dim3(grid), dim3(64), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_render<C, ST, R, 4>), dim3(grid), dim3(64), 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_render<C, ST, R, 5>), dim3(grid), dim3(64), 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_render<C, ST, R, 6>), dim3(grid), dim3(64), 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_render<C, ST, R, 7>), dim3(grid), dim3(64), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Instantiates the kernels of C channels for both storage types and both
// geometry precisions.
template <int C>
hipError_t launch_render_dispatch(const RenderLaunch& r, const RArgs& a, unsigned grid, hipStream_t st) {
    const bool bf16 = r.storage == ART_BF16;
    if (r.fp32) return bf16 ? launch_render_mode<C, 1, float>(r, a, grid, st) : launch_render_mode<C, 0, float>(r, a, grid, st);
    return bf16 ? launch_render_mode<C, 1, double>(r, a, grid, st) : launch_render_mode<C, 0, double>(r, a, grid, st);
}

}  // namespace art
