// C ABI entry points of libartemis (declared in include/artemis.h).
//
// Host code only: argument checks, device buffers, and the per-pose pipeline
//   fk (all poses, FP64)
//   per pose: skin -> radix sort -> unique/bricks/FLUT permute
//             per view group: tile binning -> render
// Every device step is one of the library's own kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "device_util.h"
#include "shade.h"
#include "internal.h"

using namespace art;

#include "render_impl.h"

namespace {

constexpr int kVersion = 10000;   // 1.0.0

art_status fail(art_ctx* ctx, art_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

art_status hip_fail(art_ctx* ctx, hipError_t e, const char* what) {
    (void)hipGetLastError();
    const art_status st = (e == hipErrorOutOfMemory) ? ART_ENOMEM : ART_EDEVICE;
    return fail(ctx, st, std::string(what) + ": " + hipGetErrorString(e));
}

struct DeviceGuard {
    int old = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

#define ART_TRY_HIP(expr, what)                          \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

bool supported_C(int C) { return C == 4 || C == 8 || C == 16 || C == 32; }

// k_accum: fold the counters of a batch of poses into the run statistics.
__global__ void k_accum(const PoseCounters* __restrict__ c, unsigned long long* __restrict__ st, uint32_t n,
                        int batch) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= batch) return;
    atomicAdd(&st[3], (unsigned long long)c[p].dropped);
    atomicAdd(&st[4], (unsigned long long)(n - c[p].dropped - c[p].M));
    atomicAdd(&st[5], (unsigned long long)c[p].nb);
}

// k_check_sigma: count the FLUT densities that are negative or not finite
// (the densities of Eq. 5-6 are non-negative) into *bad.  The compositing
// kernel reads the count and renders nothing when it is not zero.
template <int ST>
__global__ __launch_bounds__(256) void k_check_sigma(const void* __restrict__ sigma, int64_t n,
                                                     unsigned long long* __restrict__ bad) {
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float v = ST == 0 ? reinterpret_cast<const float*>(sigma)[i]
                                : bf16_to_f32(reinterpret_cast<const uint16_t*>(sigma)[i]);
        cnt += (v >= 0.0f && v <= 3.402823466e38f) ? 0u : 1u;   // false for NaN
    }
    const unsigned w = wave_sum(cnt);
    if (lane_id() == 0 && w) atomicAdd(bad, (unsigned long long)w);
}

hipError_t launch_check_sigma(const void* sigma, int storage, int64_t n, unsigned long long* bad, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    if (storage) hipLaunchKernelGGL(k_check_sigma<1>, dim3((unsigned)blocks), dim3(256), 0, st, sigma, n, bad);
    else hipLaunchKernelGGL(k_check_sigma<0>, dim3((unsigned)blocks), dim3(256), 0, st, sigma, n, bad);
    return hipGetLastError();
}

struct CallPlan {
    int C = 0;
    int storage = 0;
    bool fp32 = false;
    int Vg = 1;           // views per group
    int ngroups = 1;
    int mbits = 0;
    bool net = false;     // proposal network inference (per-item intervals)
};

art_status check_build_state(art_ctx* ctx) {
    if (ctx->n <= 0) return fail(ctx, ART_ESTATE, "no octree loaded (art_load_octree)");
    if (!ctx->has_skin) return fail(ctx, ART_ESTATE, "no skin weights (art_set_skin)");
    if (ctx->J <= 0) return fail(ctx, ART_ESTATE, "no skeleton (art_set_skeleton)");
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    if (ctx->max_bone >= ctx->J)
        return fail(ctx, ART_EINVAL, "skin bone id " + std::to_string(ctx->max_bone) +
                                         " >= number of joints " + std::to_string(ctx->J));
    return ART_OK;
}

art_status check_render_state(art_ctx* ctx) {
    art_status rc = check_build_state(ctx);
    if (rc != ART_OK) return rc;
    if (ctx->V <= 0) return fail(ctx, ART_ESTATE, "no cameras (art_set_cameras)");
    return ART_OK;
}

art_status plan_call(art_ctx* ctx, int C, art_dtype dtype, unsigned flags, CallPlan* pl) {
    if (!supported_C(C)) return fail(ctx, ART_EUNSUPPORTED, "C must be 4, 8, 16 or 32");
    if (dtype != ART_F32 && dtype != ART_BF16) return fail(ctx, ART_EINVAL, "dtype must be ART_F32 or ART_BF16");
    if (flags & ~(ART_GEOM_FP32 | ART_TIMING | ART_ASYNC)) return fail(ctx, ART_EINVAL, "unknown flag bits");
    if ((flags & ART_ASYNC) && (flags & ART_TIMING))
        return fail(ctx, ART_EINVAL, "ART_ASYNC and ART_TIMING exclude each other");
    pl->C = C;
    pl->storage = dtype == ART_BF16 ? 1 : 0;
    pl->fp32 = (flags & ART_GEOM_FP32) != 0;
    int Vg = ctx->V;
    int mbits = 0;
    while (Vg > 1 && bin_key_bits(Vg, ctx->H, ctx->W, ctx->depth, &mbits) > 32) Vg = (Vg + 1) / 2;
    if (bin_key_bits(Vg, ctx->H, ctx->W, ctx->depth, &mbits) > 32)
        return fail(ctx, ART_EUNSUPPORTED, "image too large for 32-bit tile keys");
    pl->Vg = Vg;
    pl->ngroups = (ctx->V + Vg - 1) / Vg;
    pl->mbits = mbits;
    return ART_OK;
}

// The context's working buffers: everything the library allocates beyond the
// copies of its inputs (scratch of the render, octree, proposal-network and
// shading calls).  art_set_memory_limit bounds their total capacity.
std::vector<DevBuf*> working_bufs(art_ctx* ctx) {
    Scratch& s = ctx->s;
    return {&ctx->B64, &ctx->B32, &ctx->Gtmp, &ctx->shade_act,
            &s.keys0, &s.keys1, &s.bmap, &s.wpref, &s.hist, &s.digit_tot, &s.blk0, &s.blk1, &s.occ_key,
            &s.occ_win, &s.brick_key, &s.brick_row, &s.brick_mask, &s.bin_cnt, &s.bin_off, &s.pk0, &s.pv0,
            &s.pk1, &s.pair_v, &s.tile_start, &s.tile_end, &s.counters, &s.stats, &s.ovf, &s.items, &s.queue,
            &s.loss, &s.redo, &s.interval, &ctx->mlp_theta, &ctx->mlp_m1, &ctx->mlp_m2, &ctx->mlp_packed, &ctx->mlp_cbias,
            &ctx->mlp_code, &ctx->mlp_S, &ctx->mlp_part, &ctx->mlp_lossp, &ctx->mlp_loss, &ctx->mlp_flag,
            &ctx->mlp_calib};
}

size_t working_bytes(art_ctx* ctx) {
    size_t t = 0;
    for (const DevBuf* b : working_bufs(ctx)) t += b->cap;
    return t;
}

art_status ensure_bufs(art_ctx* ctx, std::initializer_list<std::pair<DevBuf*, size_t>> req) {
    for (auto& r : req) {
        const size_t cap = r.first->cap;
        if (ctx->mem_limit > 0 && r.second > cap) {
            // growing this buffer frees its old storage and allocates max(bytes, 256)
            const size_t held = working_bytes(ctx);
            const size_t after = (held >= cap ? held - cap : 0) + std::max<size_t>(r.second, 256);
            if (after > ctx->mem_limit)
                return fail(ctx, ART_ENOMEM, "working memory would reach " + std::to_string(after) +
                                                 " bytes, above the limit of " + std::to_string(ctx->mem_limit));
        }
        ART_TRY_HIP(r.first->ensure(r.second), "device allocation");
        if (r.first->cap != cap) ctx->memo.valid = false;   // a reallocated buffer lost its contents
    }
    return ART_OK;
}

// Device memory held for the posed octrees of one batch of poses (48 GiB by
// default, ARTEMIS_SLOT_BUDGET_MB overrides); the poses of a call are processed
// in batches that fit it.
size_t slot_budget_bytes(const art_ctx* ctx) {
    size_t b = (size_t)48 << 30;
    const char* e = getenv("ARTEMIS_SLOT_BUDGET_MB");
    if (e && *e) {
        const long long mb = atoll(e);
        if (mb > 0) b = (size_t)mb << 20;
    }
    // under a working-memory limit the batches shrink to fit it
    if (ctx->mem_limit > 0) b = std::min(b, ctx->mem_limit);
    return b;
}

// Whether the adjoint merges the gradient records of one leaf before adding
// them (ARTEMIS_ADJ_MERGE = 0 never, 1 always; by default when the launch has
// at least two tiles per workgroup).
int adj_merge_policy() {
    const char* e = getenv("ARTEMIS_ADJ_MERGE");
    if (e && *e == '0') return 0;
    if (e && *e == '1') return 1;
    return 2;
}

// Whether the shading network's 1x1 head runs in its last convolution
// (ARTEMIS_SHADE_HEAD=0: a kernel of its own after it).
static bool fused_shading_head() {
    const char* e = getenv("ARTEMIS_SHADE_HEAD");
    return !(e && *e == '0');
}

// Whether the compositing kernel writes the forward maps' background pixels
// (ARTEMIS_BG_KERNEL=1: a kernel of its own before the compositing kernel).
bool bg_in_render_enabled() {
    const char* e = getenv("ARTEMIS_BG_KERNEL");
    return !(e && *e == '1');
}

// Initial capacity of one (pose, view group) tile list (ARTEMIS_PAIR_CAP
// overrides; the capacity grows when a list overflows).
size_t initial_pair_cap(size_t tiles_g) {
    const char* e = getenv("ARTEMIS_PAIR_CAP");
    if (e && *e) {
        const long long v = atoll(e);
        if (v > 0) return (size_t)v;
    }
    return std::max<size_t>((size_t)1 << 20, 16 * tiles_g);
}

size_t slot_bytes(const art_ctx* ctx, const CallPlan& pl, size_t pair_cap) {
    const size_t n = (size_t)ctx->n;
    const size_t es = pl.storage ? 2 : 4;
    const size_t tiles = (size_t)ctx->V * ((ctx->W + 7) / 8) * ((ctx->H + 7) / 8);
    // octree slot + per-leaf keys and rows + brick bitmap + bin counts + tile lists and their sort
    // scratch + tile ranges
    return n * (4 + 4 + 4 + 4 + 64) + n * 8 + (size_t)brick_words(ctx->depth) * 8 + n * pl.Vg * 8 +
           (size_t)pl.ngroups * pair_cap * 8 + pair_cap * 8 + tiles * 12 + (size_t)pl.ngroups * 9 +
           (pl.net ? tiles * 64 * 8 : 0);
}

// Sort / scan scratch and the per-slot arrays of `slots` poses.
art_status ensure_scratch(art_ctx* ctx, const CallPlan& pl, int slots) {
    Scratch& s = ctx->s;
    const size_t n = (size_t)ctx->n;
    const size_t es = pl.storage ? 2 : 4;
    const size_t V = (size_t)std::max(ctx->V, 1);
    const size_t tiles = V * ((ctx->W + 7) / 8) * ((ctx->H + 7) / 8);
    const size_t tiles_g = (size_t)pl.Vg * ((ctx->W + 7) / 8) * ((ctx->H + 7) / 8);
    if (s.pair_cap == 0) s.pair_cap = initial_pair_cap(tiles_g);
    const size_t S = (size_t)slots;
    const size_t nblk = (size_t)std::max(kScanBlocks, kUniqueBlocks);
    s.bin_stride = n * pl.Vg;
    art_status rc = ensure_bufs(ctx, {
        {&s.keys0, S * n * 4}, {&s.keys1, S * n * 4},
        {&s.bmap, S * brick_words(ctx->depth) * 4}, {&s.wpref, S * brick_words(ctx->depth) * 4},
        {&s.hist, S * 256 * (size_t)kSortBlocks * 4}, {&s.digit_tot, S * 256 * 4},
        {&s.blk0, S * nblk * 4}, {&s.blk1, S * nblk * 4},
        {&s.counters, S * sizeof(PoseCounters)}, {&s.stats, 16 * sizeof(unsigned long long)},
        {&ctx->B64, (size_t)ctx->P * ctx->J * 12 * 8}, {&ctx->B32, (size_t)ctx->P * ctx->J * 12 * 4},
        {&ctx->Gtmp, (size_t)ctx->P * ctx->J * 12 * 8},
        {&s.occ_key, S * n * 4}, {&s.occ_win, S * n * 4},
        {&s.brick_key, S * n * 4}, {&s.brick_row, S * (n + 1) * 4}, {&s.brick_mask, S * n * 64},
        {&s.bin_cnt, S * n * pl.Vg * 4}, {&s.bin_off, S * n * pl.Vg * 4},
        {&s.pk0, S * s.pair_cap * 4}, {&s.pk1, S * s.pair_cap * 4}, {&s.pv0, S * pl.ngroups * s.pair_cap * 4},
        {&s.pair_v, S * pl.ngroups * s.pair_cap * 4},
        {&s.redo, S * pl.ngroups},
        {&s.tile_start, S * tiles * 4}, {&s.tile_end, S * tiles * 4},
        {&s.ovf, S * pl.ngroups * 2 * 4},
        {&s.items, S * tiles * 4}, {&s.queue, 64}, {&s.loss, 8},
        {&s.interval, pl.net ? S * tiles * 64 * 8 : 0},
    });
    if (rc == ART_OK) s.slots = std::max(s.slots, slots);
    return rc;
}

OctreeSlot octree_slot(art_ctx* ctx, const CallPlan& pl, int slot) {
    Scratch& s = ctx->s;
    const size_t n = (size_t)ctx->n;
    const size_t es = pl.storage ? 2 : 4;
    OctreeSlot o;
    o.occ_key = s.occ_key.as<uint32_t>() + (size_t)slot * n;
    o.occ_win = s.occ_win.as<uint32_t>() + (size_t)slot * n;
    o.brick_key = s.brick_key.as<uint32_t>() + (size_t)slot * n;
    o.brick_row = s.brick_row.as<uint32_t>() + (size_t)slot * (n + 1);
    o.brick_mask = s.brick_mask.as<uint32_t>() + (size_t)slot * n * 16;
    return o;
}

struct Timing {
    bool on = false;
    std::vector<hipEvent_t>* pool = nullptr;   // the context's events, created once and reused
    size_t used = 0;
    std::vector<int> stage;   // stage id of the interval ending at event i
    void record(hipStream_t st, int stage_id) {
        if (!on || !pool) return;
        if (used == pool->size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            pool->push_back(e);
        }
        (void)hipEventRecord((*pool)[used++], st);
        stage.push_back(stage_id);
    }
    void finish(art_ctx* ctx) {
        for (int i = 0; i < 7; ++i) ctx->timing_ms[i] = 0.0f;
        ctx->timing_nrender = 0;
        for (size_t i = 1; i < used; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, (*pool)[i - 1], (*pool)[i]) == hipSuccess && stage[i] >= 0) {
                ctx->timing_ms[stage[i]] += ms;
                if (stage[i] == 4) ctx->timing_nrender++;
            }
        }
        if (used >= 2) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, (*pool)[0], (*pool)[used - 1]) == hipSuccess) ctx->timing_ms[5] = ms;
        }
        ctx->timing_valid = on;
        used = 0;
        stage.clear();
    }
};

struct PassOut {
    // forward
    float* out_feat = nullptr;
    float* out_alpha = nullptr;
    float* out_tfinal = nullptr;
    // backward
    const float* fwd_feat = nullptr;
    const float* fwd_tfinal = nullptr;
    const float* d_feat = nullptr;
    const float* d_alpha = nullptr;
    float* d_sigma = nullptr;
    float* d_leaf_feat = nullptr;
    // proposal: labels (mode 3) / intervals, margin and F2 threshold (mode 4)
    float* labels = nullptr;
    const float* intervals = nullptr;
    float margin = 0.0f;
    float f2_tau = -1.0f;
    bool near_only = false;
    // depth buffer (mode 5)
    float* out_depth = nullptr;
    float depth_sigma = 0.0f;
    // view-dependent features (mode 6)
    int sh_H = 1;
    // debug
    int max_hits = 0;
    int debug_view = 0;
    int32_t* hit_leaf = nullptr;
    double* hit_delta = nullptr;
    int32_t* hit_count = nullptr;
    bool single_pose = false;   // maps hold one pose only
    bool reuse = false;         // ART_REUSE_BUILD was asked for
    // ray checkpoints (mode 7 writes them, the segmented adjoint reads them)
    float* ckpt = nullptr;
    int32_t* ckpt_n = nullptr;
    int ckpt_K = 0, ckpt_every = 0;
};

// Skinning + octree build of poses [p0, p0 + batch) into slots 0..batch-1.
// cell_keys: also store the posed key of each occupied cell (occ_key), which
// only the inspection call reads.
art_status build_batch(art_ctx* ctx, const CallPlan& pl, int p0, int batch, const void* sigma, const void* feat,
                       int* launches, Timing& tm, bool cell_keys = false) {
    Scratch& s = ctx->s;
    hipStream_t st = ctx->stream;
    PoseCounters* cnt = s.counters.as<PoseCounters>();
    const size_t n = (size_t)ctx->n;
    ctx->memo.valid = false;   // the slots are overwritten
    tm.record(st, -1);
    ART_TRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), 0u, (size_t)batch * sizeof(PoseCounters) / 4, st),
                "fill");
    const uint32_t bwords = brick_words(ctx->depth);
    ART_TRY_HIP(launch_fill_u32(s.bmap.as<uint32_t>(), 0u, (size_t)batch * bwords, st), "fill");
    ART_TRY_HIP(launch_skin(ctx->ijk.as<uint16_t>(), ctx->bone.as<uint8_t>(), ctx->weight.as<float>(), ctx->n,
                            ctx->depth, ctx->B64.as<double>() + (size_t)p0 * ctx->J * 12,
                            ctx->B32.as<float>() + (size_t)p0 * ctx->J * 12, ctx->J, pl.fp32, batch,
                            s.keys0.as<uint32_t>(), nullptr, s.bmap.as<uint32_t>(), bwords, cnt, st),
                "skin");
    *launches += 3;
    tm.record(st, 1);
    OctreeSlot os = octree_slot(ctx, pl, 0);
    if (!cell_keys) os.occ_key = nullptr;
    ART_TRY_HIP(launch_build_octree_dense(s.keys0.as<uint32_t>(), (uint32_t)n, ctx->depth, s, os, batch, st,
                                          launches),
                "octree build");
    hipLaunchKernelGGL(k_accum, dim3((batch + 63) / 64), dim3(64), 0, st, (const PoseCounters*)cnt,
                       s.stats.as<unsigned long long>(), (uint32_t)n, batch);
    *launches += 1;
    tm.record(st, 2);
    return ART_OK;
}

// Build every pose of the batch [p0, p0 + Pb) into its slot and bin its view
// groups into tile lists.  `redo` (indexed by slot * ngroups + group) marks the
// (pose, group) items whose tile lists overflowed in an earlier attempt.
art_status build_and_bin(art_ctx* ctx, const CallPlan& pl, int p0, int Pb, const void* sigma, const void* feat,
                         const std::vector<char>* redo, int* launches, Timing& tm) {
    Scratch& s = ctx->s;
    hipStream_t st = ctx->stream;
    const size_t TPV = (size_t)((ctx->W + 7) / 8) * ((ctx->H + 7) / 8);
    art_status rc = build_batch(ctx, pl, p0, Pb, sigma, feat, launches, tm);
    if (rc != ART_OK) return rc;
    const uint8_t* redo_dev = nullptr;
    if (redo) {
        std::vector<uint8_t> m(redo->begin(), redo->end());
        ART_TRY_HIP(hipMemcpyAsync(s.redo.p, m.data(), m.size(), hipMemcpyHostToDevice, st), "copy");
        ART_TRY_HIP(hipStreamSynchronize(st), "copy");
        redo_dev = s.redo.as<uint8_t>();
    }
    tm.record(st, -1);
    ART_TRY_HIP(launch_fill_u32(s.tile_start.as<uint32_t>(), 0u, (size_t)Pb * ctx->V * TPV, st), "fill");
    ART_TRY_HIP(launch_fill_u32(s.tile_end.as<uint32_t>(), 0u, (size_t)Pb * ctx->V * TPV, st), "fill");
    *launches += 2;
    const OctreeSlot os = octree_slot(ctx, pl, 0);
    for (int gi = 0; gi < pl.ngroups; ++gi) {
        const int v0 = gi * pl.Vg;
        const int Vg = std::min(ctx->V, v0 + pl.Vg) - v0;
        ART_TRY_HIP(launch_bin(s, ctx->cam.as<CamParams>(), os, (size_t)ctx->n, Pb, ctx->V, v0, Vg, gi, pl.ngroups,
                               ctx->H, ctx->W, ctx->depth, pl.fp32, st, launches),
                    "tile binning");
        hipLaunchKernelGGL(k_pairs, dim3((Pb + 63) / 64), dim3(64), 0, st, (const PoseCounters*)s.counters.as<PoseCounters>(),
                           s.stats.as<unsigned long long>(), s.ovf.as<uint32_t>(), pl.ngroups, gi, redo_dev, Pb);
        *launches += 1;
    }
    return ART_OK;
}

// One batch of poses [p0, p1): build every pose into its slot, bin its view
// groups (both skipped when `reuse`: the slots already hold this batch's
// octrees and tile lists), then render all (pose, view) maps of the batch in
// one launch.  `redo` restricts the render to the items that overflowed.
art_status run_batch(art_ctx* ctx, const CallPlan& pl, int mode, float lambda, const void* sigma,
                     const void* feat, const PassOut& o, int p0, int p1,
                     const std::vector<char>* redo, int* launches, Timing& tm, bool reuse = false) {
    Scratch& s = ctx->s;
    hipStream_t st = ctx->stream;
    const int Pb = p1 - p0;
    const size_t TPV = (size_t)((ctx->W + 7) / 8) * ((ctx->H + 7) / 8);
    if (!reuse) {
        art_status rc = build_and_bin(ctx, pl, p0, Pb, sigma, feat, redo, launches, tm);
        if (rc != ART_OK) return rc;
    }
    tm.record(st, 3);
    tm.record(st, -1);
    RenderLaunch r{};
    r.C = pl.C;
    r.storage = pl.storage ? ART_BF16 : ART_F32;
    r.fp32 = pl.fp32;
    r.mode = mode;
    r.depth = ctx->depth;
    r.Pb = Pb;
    r.V = ctx->V;
    r.H = ctx->H;
    r.W = ctx->W;
    r.Vg = pl.Vg;
    r.ngroups = pl.ngroups;
    r.ncap = (uint32_t)ctx->n;
    r.lambda = lambda;
    r.cam = ctx->cam.as<CamParams>();
    r.s = &ctx->s;
    r.sigma = sigma;
    r.feat = feat;
    const size_t HW = (size_t)ctx->H * ctx->W;
    const size_t m0 = o.single_pose ? 0 : (size_t)p0 * ctx->V;   // first map of the batch
    if (o.out_feat) r.out_feat = o.out_feat + m0 * pl.C * HW;
    if (o.out_alpha) r.out_alpha = o.out_alpha + m0 * HW;
    if (o.out_tfinal) r.out_tfinal = o.out_tfinal + m0 * HW;
    if (o.ckpt) {
        r.ckpt = o.ckpt + m0 * HW * (size_t)o.ckpt_K * (pl.C + 4);
        r.ckpt_n = o.ckpt_n + m0 * HW;
        r.ckpt_K = o.ckpt_K;
        r.ckpt_every = o.ckpt_every;
    }
    if (o.fwd_feat) r.fwd_feat = o.fwd_feat + m0 * pl.C * HW;
    if (o.fwd_tfinal) r.fwd_tfinal = o.fwd_tfinal + m0 * HW;
    if (o.d_feat) r.d_feat = o.d_feat + m0 * pl.C * HW;
    if (o.d_alpha) r.d_alpha = o.d_alpha + m0 * HW;
    r.d_sigma = o.d_sigma;
    r.d_leaf_feat = o.d_leaf_feat;
    if (o.labels) r.labels = o.labels + m0 * HW * 2;
    if (o.intervals) r.interval = o.intervals + m0 * HW * 2;
    r.margin = o.margin;
    r.f2_tau = o.f2_tau;
    r.near_only = o.near_only;
    if (o.out_depth) r.out_depth = o.out_depth + m0 * HW;
    r.depth_sigma = o.depth_sigma;
    r.sh_H = o.sh_H;
    r.J = ctx->J;
    r.dom_bone = ctx->dom_bone.as<uint8_t>();
    r.bone_rot = ctx->B32.as<float>() + (size_t)p0 * ctx->J * 12;
    r.max_hits = o.max_hits;
    r.debug_view = o.debug_view;
    r.hit_leaf = o.hit_leaf;
    r.hit_delta = o.hit_delta;
    r.hit_count = o.hit_count;
    int side = 1;
    while (side < (ctx->W + 7) / 8 || side < (ctx->H + 7) / 8) side <<= 1;
    TileLaunch tl{};
    tl.Pb = Pb;
    tl.V = ctx->V;
    tl.Vg = pl.Vg;
    tl.ngroups = pl.ngroups;
    tl.H = ctx->H;
    tl.W = ctx->W;
    tl.C = pl.C;
    tl.tiles_pow4 = (uint32_t)(side * side);
    tl.debug_view = mode == 2 ? o.debug_view : -1;
    tl.ovf = s.ovf.as<uint32_t>();
    tl.tile_start = s.tile_start.as<uint32_t>();
    tl.tile_end = s.tile_end.as<uint32_t>();
    tl.items = s.items.as<uint32_t>();
    tl.counters = s.queue.as<uint32_t>();
    tl.out_feat = r.out_feat;
    tl.out_alpha = r.out_alpha;
    tl.out_tfinal = r.out_tfinal;
    tl.labels = r.labels;
    tl.out_depth = r.out_depth;
    tl.hit_count = r.hit_count;
    tl.stats = s.stats.as<unsigned long long>();
    // the forward maps' background pixels are written by the compositing
    // kernel's waves between their tiles (overlapping their compositing)
    tl.bg_in_render = (mode == 0 || mode == 4 || mode == 5 || mode == 6 || mode == 7) && tl.out_feat && !tl.labels &&
                      !tl.hit_count && background_vectorised(tl) && bg_in_render_enabled() &&
                      (uint64_t)Pb * ctx->V * ctx->H * ctx->W / 4 < (1ull << 31);
    r.bg_in_render = tl.bg_in_render;
    ART_TRY_HIP(launch_tiles(tl, st), "tile compaction");
    *launches += ((r.out_feat || r.hit_count || r.labels) && !tl.bg_in_render) ? 3 : 2;
    tm.record(st, 3);
    if (mode == 4 && !o.intervals) {   // proposal network: intervals of the rays of every non-empty tile
        InferLaunch ia{};
        ia.packed = ctx->mlp_packed.as<uint16_t>();
        ia.theta = ctx->mlp_theta.as<float>();
        ia.cbias = ctx->mlp_cbias.as<float>();
        ia.m = mlp_dims(ctx->J);
        ia.cam = ctx->cam.as<CamParams>();
        ia.items = s.items.as<uint32_t>();
        ia.n_items = s.queue.as<uint32_t>();
        ia.V = ctx->V;
        ia.TX = (ctx->W + 7) / 8;
        ia.TPV = (int)TPV;
        ia.pose0 = p0;
        ia.out = s.interval.as<float>();
        ART_TRY_HIP(launch_mlp_infer_tiles(ia, (unsigned)num_cus() * 8u, st), "proposal inference");
        *launches += 1;
        r.interval = s.interval.as<float>();
        r.interval_by_item = true;
        tm.record(st, 6);
    }
    ART_TRY_HIP(launch_render(r, st), "render");
    *launches += 1;
    tm.record(st, 4);
    return ART_OK;
}

// Pose codes of the current poses, BF16 operands and per-pose biases of the
// current proposal weights.
art_status mlp_prepare(art_ctx* ctx) {
    if (ctx->mlp_J <= 0 || ctx->mlp_J != ctx->J)
        return fail(ctx, ART_ESTATE, "no proposal weights for the current skeleton (art_proposal_set_weights)");
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    const MlpDims m = mlp_dims(ctx->J);
    hipStream_t st = ctx->stream;
    art_status rc = ensure_bufs(ctx, {{&ctx->mlp_code, (size_t)ctx->P * 6 * ctx->J * 4},
                                      {&ctx->mlp_packed, (size_t)mlp_packed_elems() * 2},
                                      {&ctx->mlp_cbias, (size_t)ctx->P * 64 * 4}});
    if (rc != ART_OK) return rc;
    if (ctx->code_version != ctx->poses_version) {
        ART_TRY_HIP(launch_pose_code(ctx->pose.as<double>(), ctx->J, ctx->P, ctx->mlp_code.as<float>(), st), "pose code");
        ctx->code_version = ctx->poses_version;
    }
    ART_TRY_HIP(launch_mlp_prep(ctx->mlp_theta.as<float>(), m, ctx->mlp_code.as<float>(), ctx->P,
                                ctx->mlp_packed.as<uint16_t>(), ctx->mlp_cbias.as<float>(), st),
                "proposal prep");
    return ART_OK;
}

// Whether the scratch slots still hold the posed octrees and tile lists of a
// whole-batch call that a call with plan `pl` can use unchanged.
bool memo_matches(const art_ctx* ctx, const CallPlan& pl) {
    const art_ctx::BuildMemo& m = ctx->memo;
    return m.valid && m.version == ctx->state_version && m.fp32 == pl.fp32 && m.P == ctx->P && m.Vg == pl.Vg &&
           m.ngroups == pl.ngroups && m.H == ctx->H && m.W == ctx->W && m.pair_cap == ctx->s.pair_cap &&
           m.occ == ctx->s.occ_win.p && m.lists == ctx->s.pair_v.p && m.rows == ctx->s.keys1.p &&
           m.tiles == ctx->s.tile_start.p && m.counters == ctx->s.counters.p;
}
void fill_memo(const art_ctx* ctx, const CallPlan& pl, art_ctx::BuildMemo& m) {
    m.valid = true;
    m.version = ctx->state_version;
    m.fp32 = pl.fp32;
    m.P = ctx->P;
    m.Vg = pl.Vg;
    m.ngroups = pl.ngroups;
    m.H = ctx->H;
    m.W = ctx->W;
    m.pair_cap = ctx->s.pair_cap;
    m.occ = ctx->s.occ_win.p;
    m.lists = ctx->s.pair_v.p;
    m.rows = ctx->s.keys1.p;
    m.tiles = ctx->s.tile_start.p;
    m.counters = ctx->s.counters.p;
}
void take_memo(art_ctx* ctx, const CallPlan& pl) { fill_memo(ctx, pl, ctx->memo); }

art_status render_call(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                       float lambda, unsigned flags, int mode, const PassOut& o, int pose_lo,
                       int pose_hi) {
    art_status rc = check_render_state(ctx);
    if (rc != ART_OK) return rc;
    CallPlan pl;
    rc = plan_call(ctx, C, dtype, flags, &pl);
    if (rc != ART_OK) return rc;
    pl.net = mode == 4 && !o.intervals;
    if (!sigma || !feat) return fail(ctx, ART_EINVAL, "sigma / feat must be device pointers");
    if (!(lambda >= 0.0f && lambda < 1.0f)) return fail(ctx, ART_EINVAL, "lambda_th must be in [0, 1)");
    const int P = pose_hi - pose_lo;
    if (ctx->s.pair_cap == 0) {
        const size_t tiles_g = (size_t)pl.Vg * ((ctx->W + 7) / 8) * ((ctx->H + 7) / 8);
        ctx->s.pair_cap = initial_pair_cap(tiles_g);
    }
    int slots = (int)std::min<size_t>((size_t)P, std::max<size_t>(1, slot_budget_bytes(ctx) / slot_bytes(ctx, pl, ctx->s.pair_cap)));
    rc = ensure_scratch(ctx, pl, slots);
    if (rc != ART_OK) return rc;
    hipStream_t st = ctx->stream;
    int launches = 0;
    Timing tm;
    tm.on = (flags & ART_TIMING) != 0;
    tm.pool = &ctx->ev_pool;
    const bool whole = pose_lo == 0 && pose_hi == ctx->P && slots >= P;   // one batch, every pose
    const bool reuse = o.reuse && whole && memo_matches(ctx, pl);
    // ART_ASYNC: nothing is read back when the poses fit one batch (otherwise
    // the slots are reused and the call stays synchronous)
    const bool async = (flags & ART_ASYNC) != 0 && slots >= P;
    ctx->async_pending = false;
    ctx->async_memo.valid = false;

    ART_TRY_HIP(launch_fill_u32(ctx->s.stats.as<uint32_t>(), 0u, 32, st), "fill");
    ART_TRY_HIP(launch_check_sigma(sigma, pl.storage, ctx->n, ctx->s.stats.as<unsigned long long>() + kStatBadSigma,
                                   st),
                "density check");
    launches += 1;
    tm.record(st, -1);
    if (!reuse) {
        ART_TRY_HIP(launch_fk(ctx->parent.as<int32_t>(), ctx->rest.as<double>(), ctx->pose.as<double>(), ctx->J,
                              ctx->P, ctx->Gtmp.as<double>(), ctx->B64.as<double>(), ctx->B32.as<float>(), st),
                    "fk");
        launches += 1;
    }
    launches += 1;
    tm.record(st, 0);
    unsigned long long hst[16] = {0};
    bool reran = false;   // some (pose, view group) items were rendered again after an overflow
    for (int p0 = pose_lo; p0 < pose_hi; p0 += slots) {
        const int p1 = std::min(pose_hi, p0 + slots);
        const size_t items = (size_t)(p1 - p0) * pl.ngroups;
        rc = run_batch(ctx, pl, mode, lambda, sigma, feat, o, p0, p1, nullptr, &launches, tm, reuse);
        if (rc != ART_OK) return rc;
        if (async) {   // art_render_status reads the overflow flags and statistics
            ctx->async_pending = true;
            ctx->async_items = items;
            ctx->async_launches = launches;
            // the slots hold every pose's octree and tile lists unless an item
            // overflowed, which only the status call can tell
            if (whole) fill_memo(ctx, pl, ctx->async_memo);
            return ART_OK;
        }
        // a (pose, view group) whose tile lists overflowed was skipped by the
        // render kernel: grow the list buffers and run those items again
        for (int attempt = 0; attempt < 3; ++attempt) {
            std::vector<uint32_t> hov(items * 2);
            ART_TRY_HIP(hipMemcpyAsync(hov.data(), ctx->s.ovf.p, items * 2 * 4, hipMemcpyDeviceToHost, st), "copy");
            // the run statistics come back with the same synchronisation (the
            // copy after the last batch's last attempt is the call's total)
            ART_TRY_HIP(hipMemcpyAsync(hst, ctx->s.stats.p, sizeof(hst), hipMemcpyDeviceToHost, st), "copy");
            ART_TRY_HIP(hipStreamSynchronize(st), "render");
            if (hst[kStatBadSigma] != 0ull)   // the compositing kernel rendered nothing
                return fail(ctx, ART_EINVAL, std::to_string(hst[kStatBadSigma]) +
                                                 " FLUT densities are negative or not finite");
            std::vector<char> redo(items, 0);
            size_t need = 0;
            bool any = false;
            for (size_t i = 0; i < items; ++i) ctx->s.pair_hint = std::max<size_t>(ctx->s.pair_hint, hov[2 * i + 1]);
            for (size_t i = 0; i < items; ++i)
                if (hov[2 * i] != 0u && hov[2 * i + 1] > ctx->s.pair_cap) {
                    redo[i] = 1;
                    any = true;
                    need = std::max<size_t>(need, hov[2 * i + 1]);
                }
            if (!any) break;
            if (attempt == 2) return fail(ctx, ART_EDEVICE, "tile list buffer overflow persisted");
            reran = true;
            ctx->s.pair_cap = need + need / 4 + 1024;
            rc = ensure_scratch(ctx, pl, slots);
            if (rc != ART_OK) return rc;
            rc = run_batch(ctx, pl, mode, lambda, sigma, feat, o, p0, p1, &redo, &launches, tm);
            if (rc != ART_OK) return rc;
        }
    }
    for (int i = 0; i < 7; ++i) ctx->stats[i] = (int64_t)hst[i];
    ctx->stats[7] = launches;
    ctx->stats[8] = (int64_t)hst[7];
    ctx->stats[9] = (int64_t)hst[8];
    ctx->stats[10] = (int64_t)hst[9];
    ctx->stats[11] = (int64_t)hst[10];
    ctx->stats[12] = (int64_t)hst[11];
    ctx->stats[13] = (int64_t)hst[12];
    ctx->stats[14] = (int64_t)hst[13];
    tm.finish(ctx);
    // the slots hold every pose's octree and tile lists - unless an overflow
    // re-run rebuilt only some items: the others' overflow flags then mark them
    // as done, and a reusing call would skip them
    if (whole && !reran) take_memo(ctx, pl);
    return ART_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// render launcher (kernel argument packing)
// ---------------------------------------------------------------------------
namespace art {
int num_cus() {
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            n_cu = prop.multiProcessorCount;
        if (n_cu <= 0) n_cu = 256;
    }
    return n_cu;
}

hipError_t launch_render(const RenderLaunch& r, hipStream_t st) {
    const Scratch& s = *r.s;
    RArgs a{};
    a.cam = r.cam;
    a.Pb = r.Pb;
    a.V = r.V;
    a.H = r.H;
    a.W = r.W;
    a.TX = (r.W + 7) / 8;
    a.TY = (r.H + 7) / 8;
    a.TPV = a.TX * a.TY;
    a.depth = r.depth;
    a.Vg = r.Vg;
    a.ngroups = r.ngroups;
    a.items = s.items.as<uint32_t>();
    a.n_items = s.queue.as<uint32_t>();
    a.queue = s.queue.as<uint32_t>() + 1;
    a.ncap = r.ncap;
    a.pair_cap = (uint32_t)s.pair_cap;
    a.lambda = r.lambda;
    a.tile_start = s.tile_start.as<uint32_t>();
    a.tile_end = s.tile_end.as<uint32_t>();
    a.pair_v = s.pair_v.as<uint32_t>();
    a.ovf = s.ovf.as<uint32_t>();
    a.brick_key = s.brick_key.as<uint32_t>();
    a.brick_row = s.brick_row.as<uint32_t>();
    a.brick_mask = s.brick_mask.as<uint32_t>();
    a.occ_win = s.occ_win.as<uint32_t>();
    a.sigma = r.sigma;
    a.feat = r.feat;
    a.out_feat = r.out_feat;
    a.out_alpha = r.out_alpha;
    a.out_tfinal = r.out_tfinal;
    a.fwd_feat = r.fwd_feat;
    a.fwd_tfinal = r.fwd_tfinal;
    a.d_feat = r.d_feat;
    a.d_alpha = r.d_alpha;
    a.d_sigma = r.d_sigma;
    a.d_leaf_feat = r.d_leaf_feat;
    a.labels = r.labels;
    a.interval = r.interval;
    a.interval_by_item = r.interval_by_item ? 1 : 0;
    a.margin = r.margin;
    a.f2_tau = r.f2_tau;
    a.near_only = r.near_only ? 1 : 0;
    a.out_depth = r.out_depth;
    a.depth_sigma = r.depth_sigma;
    a.sh_H = r.sh_H;
    a.J = r.J;
    a.dom_bone = r.dom_bone;
    a.bone_rot = r.bone_rot;
    a.adj_merge = adj_merge_policy();
    a.ckpt = r.ckpt;
    a.ckpt_n = r.ckpt_n;
    a.ckpt_K = r.ckpt_K;
    a.ckpt_every = r.ckpt ? r.ckpt_every : 0;
    a.bg_in_render = r.bg_in_render ? 1 : 0;
    a.max_hits = r.max_hits;
    a.debug_view = r.debug_view;
    a.hit_leaf = r.hit_leaf;
    a.hit_delta = r.hit_delta;
    a.hit_count = r.hit_count;
    a.stats = s.stats.as<unsigned long long>();
    // persistent single-wave workgroups: about two per resident slot
    const unsigned grid = (unsigned)num_cus() * 32u;
    switch (r.C) {
        case 4: return launch_render_c<4>(r, a, grid, st);
        case 8: return launch_render_c<8>(r, a, grid, st);
        case 16: return launch_render_c<16>(r, a, grid, st);
        case 32: return launch_render_c<32>(r, a, grid, st);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace art

// ---------------------------------------------------------------------------
// Shading network ("Light" U-Net) layer table
// ---------------------------------------------------------------------------
namespace art {
struct ShadeLayer {
    int cin_a, cin_b, cout;   // channels from the same-resolution source, from the upsampled one, out
};
// Encoder levels of 32, 64, 128 and 256 channels (two 3x3 convolutions each,
// 2x2 max pooling between levels); decoder levels 128, 64, 32 whose first
// convolution reads [skip connection, nearest-upsampled deeper level]; a 1x1
// head to RGB + opacity.  Layer 0's input width is the feature width C.
constexpr int kShadeLayers = 14;
constexpr ShadeLayer kShade[kShadeLayers] = {
    {0, 0, 32},    {32, 0, 32},                       // level 0 (cin of layer 0 = C)
    {32, 0, 64},   {64, 0, 64},                       // level 1
    {64, 0, 128},  {128, 0, 128},                     // level 2
    {128, 0, 256}, {256, 0, 256},                     // level 3
    {128, 256, 128}, {128, 0, 128},                   // decoder level 2
    {64, 128, 64},   {64, 0, 64},                     // decoder level 1
    {32, 64, 32},    {32, 0, 32},                     // decoder level 0
};
inline int shade_cin(int l, int C) { return l == 0 ? C : kShade[l].cin_a + kShade[l].cin_b; }
inline int shade_cin_pad(int l) { return l == 0 ? 32 : kShade[l].cin_a + kShade[l].cin_b; }

// Activation buffers of the network for HW level-0 pixels (halves, each
// buffer 256-byte aligned): level 0: X, T0, E0 (32 ch); level 1: P0 (32), T1,
// E1 (64); level 2: P1 (64), T2, E2 (128); level 3: P2 (128), T3, B (256).
// 166 halves per pixel in all.
constexpr int kShadeBufs = 12;
inline size_t shade_layout(size_t HW, size_t off[kShadeBufs]) {
    const size_t sz[kShadeBufs] = {HW * 32, HW * 32, HW * 32, HW / 4 * 32, HW / 4 * 64, HW / 4 * 64,
                                   HW / 16 * 64, HW / 16 * 128, HW / 16 * 128, HW / 64 * 128, HW / 64 * 256,
                                   HW / 64 * 256};
    size_t tot = 0;
    for (int i = 0; i < kShadeBufs; ++i) {
        off[i] = tot;
        tot += (sz[i] + 127) / 128 * 128;
    }
    return tot;
}
}  // namespace art

// Fixed activation array of art_shading_forward_noalloc: every GPU the library
// runs on holds one copy from the code object's load until the process ends.
// In host code `scratch` is only a stand-in for the symbol: its device address
// on each GPU comes from hipGetSymbolAddress (fixed_scratch_address), and only
// that address is passed to kernels.
static __device__ __align__(256) uint16_t scratch[ART_SHADING_NOALLOC_BYTES / 2];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed_addr[kMaxDevices] = {};

// Device address of the fixed array on `device`, resolved once per device with
// that device current.
hipError_t fixed_scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    if (!g_fixed_addr[device]) {
        DeviceGuard g(device);
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_fixed_addr[device] = p;
    }
    *out = g_fixed_addr[device];
    return hipSuccess;
}
}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

int art_version(void) { return kVersion; }

art_status art_create(int device, void* stream, art_ctx** out) {
    if (!out) return ART_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return ART_EDEVICE;
    }
    if (device < 0 || device >= count) return ART_EINVAL;
    void* fixed = nullptr;
    if (fixed_scratch_address(device, &fixed) != hipSuccess) {
        (void)hipGetLastError();
        return ART_EDEVICE;
    }
    art_ctx* ctx = new (std::nothrow) art_ctx();
    if (!ctx) return ART_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->shade_fixed = fixed;
    *out = ctx;
    return ART_OK;
}

void art_destroy(art_ctx* ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        else (void)hipDeviceSynchronize();
        for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
        DevBuf* bufs[] = {&ctx->ijk, &ctx->bone, &ctx->weight, &ctx->dom_bone, &ctx->shade_w, &ctx->shade_b,
                          &ctx->shade_head, &ctx->shade_act, &ctx->parent, &ctx->rest, &ctx->pose,
                          &ctx->cam, &ctx->B64, &ctx->B32, &ctx->Gtmp,
                          &ctx->s.keys0, &ctx->s.keys1, &ctx->s.bmap, &ctx->s.wpref, &ctx->s.hist,
                          &ctx->s.digit_tot, &ctx->s.blk0, &ctx->s.blk1, &ctx->s.occ_key, &ctx->s.occ_win,
                          &ctx->s.brick_key, &ctx->s.brick_row, &ctx->s.brick_mask, &ctx->s.bin_cnt, &ctx->s.bin_off, &ctx->s.pk0, &ctx->s.pv0,
                          &ctx->s.pk1, &ctx->s.pair_v, &ctx->s.tile_start, &ctx->s.tile_end,
                          &ctx->s.counters, &ctx->s.stats, &ctx->s.ovf, &ctx->s.items, &ctx->s.queue, &ctx->s.loss,
                          &ctx->s.redo, &ctx->s.interval, &ctx->mlp_theta, &ctx->mlp_m1, &ctx->mlp_m2,
                          &ctx->mlp_packed, &ctx->mlp_cbias, &ctx->mlp_code, &ctx->mlp_S, &ctx->mlp_part,
                          &ctx->mlp_lossp, &ctx->mlp_loss, &ctx->mlp_flag, &ctx->mlp_calib};
        for (DevBuf* b : bufs) b->release();
    }
    delete ctx;
}

const char* art_last_error(const art_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

uint64_t art_state_version(const art_ctx* ctx) { return ctx ? ctx->state_version : 0; }

art_status art_set_memory_limit(art_ctx* ctx, int64_t bytes) {
    if (!ctx) return ART_EINVAL;
    ctx->mem_limit = bytes > 0 ? (size_t)bytes : 0;
    return ART_OK;
}

art_status art_get_memory(art_ctx* ctx, int64_t* working_bytes_out, int64_t* limit_out) {
    if (!ctx) return ART_EINVAL;
    if (working_bytes_out) *working_bytes_out = (int64_t)working_bytes(ctx);
    if (limit_out) *limit_out = (int64_t)ctx->mem_limit;
    return ART_OK;
}

art_status art_load_octree(art_ctx* ctx, int depth, int64_t n, const uint16_t* ijk) {
    if (!ctx) return ART_EINVAL;
    ctx->state_version++;   // posed octrees and tile lists of earlier calls no longer apply
    {
        const std::string err = check_octree(depth, n, ijk);
        if (!err.empty()) return fail(ctx, ART_EINVAL, err);
    }
    DeviceGuard g(ctx->device);
    DevBuf nb;
    ART_TRY_HIP(nb.ensure((size_t)n * 3 * 2), "device allocation");
    hipError_t e = hipMemcpy(nb.p, ijk, (size_t)n * 3 * 2, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        nb.release();
        return hip_fail(ctx, e, "copy");
    }
    ctx->ijk.release();
    ctx->ijk = nb;
    ctx->depth = depth;
    ctx->n = n;
    ctx->has_skin = false;
    ctx->max_bone = -1;
    ctx->bone.release();
    ctx->weight.release();
    return ART_OK;
}

art_status art_set_skin(art_ctx* ctx, const uint8_t* bone, const float* weight) {
    if (!ctx) return ART_EINVAL;
    ctx->state_version++;   // posed octrees and tile lists of earlier calls no longer apply
    if (ctx->n <= 0) return fail(ctx, ART_ESTATE, "no octree loaded (art_load_octree)");
    const size_t n = (size_t)ctx->n;
    int mb = -1;
    // the bone of each leaf's largest weight (the first of equal ones) stands
    // for the leaf's rotation in the view-dependent features
    std::vector<uint8_t> dom;
    {
        const std::string err = check_skin(ctx->n, bone, weight, &mb, &dom);
        if (!err.empty()) return fail(ctx, ART_EINVAL, err);
    }
    DeviceGuard g(ctx->device);
    DevBuf b, w, db;
    ART_TRY_HIP(b.ensure(4 * n), "device allocation");
    hipError_t e = w.ensure(4 * n * 4);
    if (e == hipSuccess) e = db.ensure(n);
    if (e != hipSuccess) {
        b.release();
        w.release();
        return hip_fail(ctx, e, "device allocation");
    }
    e = hipMemcpy(b.p, bone, 4 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.p, weight, 4 * n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(db.p, dom.data(), n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        b.release();
        w.release();
        db.release();
        return hip_fail(ctx, e, "copy");
    }
    ctx->bone.release();
    ctx->weight.release();
    ctx->dom_bone.release();
    ctx->bone = b;
    ctx->weight = w;
    ctx->dom_bone = db;
    ctx->has_skin = true;
    ctx->max_bone = mb;
    return ART_OK;
}

art_status art_set_skeleton(art_ctx* ctx, int J, const int32_t* parent, const double* rest_joint) {
    if (!ctx) return ART_EINVAL;
    ctx->state_version++;   // posed octrees and tile lists of earlier calls no longer apply
    {
        const std::string err = check_skeleton(J, parent, rest_joint);
        if (!err.empty()) return fail(ctx, ART_EINVAL, err);
    }
    DeviceGuard g(ctx->device);
    DevBuf pb, rb;
    ART_TRY_HIP(pb.ensure((size_t)J * 4), "device allocation");
    hipError_t e = rb.ensure((size_t)J * 24);
    if (e == hipSuccess) e = hipMemcpy(pb.p, parent, (size_t)J * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(rb.p, rest_joint, (size_t)J * 24, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pb.release();
        rb.release();
        return hip_fail(ctx, e, "skeleton upload");
    }
    ctx->parent.release();
    ctx->rest.release();
    ctx->parent = pb;
    ctx->rest = rb;
    if (J != ctx->J) {   // poses no longer match the skeleton
        ctx->P = 0;
        ctx->pose.release();
    }
    ctx->J = J;
    return ART_OK;
}

art_status art_set_poses(art_ctx* ctx, int P, const double* r, const double* R, const double* T) {
    if (!ctx) return ART_EINVAL;
    ctx->state_version++;   // posed octrees and tile lists of earlier calls no longer apply
    if (ctx->J <= 0) return fail(ctx, ART_ESTATE, "no skeleton (art_set_skeleton)");
    std::vector<double> buf;
    {
        const std::string err = pack_poses(ctx->J, P, r, R, T, &buf);
        if (!err.empty()) return fail(ctx, ART_EINVAL, err);
    }
    DeviceGuard g(ctx->device);
    DevBuf pb;
    ART_TRY_HIP(pb.ensure(buf.size() * 8), "device allocation");
    hipError_t e = hipMemcpy(pb.p, buf.data(), buf.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pb.release();
        return hip_fail(ctx, e, "copy");
    }
    ctx->pose.release();
    ctx->pose = pb;
    ctx->P = P;
    ctx->poses_version++;
    return ART_OK;
}

art_status art_set_cameras(art_ctx* ctx, int V, int H, int W, const double* K, const double* c2w) {
    if (!ctx) return ART_EINVAL;
    ctx->state_version++;   // posed octrees and tile lists of earlier calls no longer apply
    std::vector<CamParams> cams;
    {
        const std::string err = check_cameras(V, H, W, K, c2w, &cams);
        if (!err.empty()) return fail(ctx, ART_EINVAL, err);
    }
    DeviceGuard g(ctx->device);
    DevBuf cb;
    ART_TRY_HIP(cb.ensure(sizeof(CamParams) * V), "device allocation");
    hipError_t e = hipMemcpy(cb.p, cams.data(), sizeof(CamParams) * V, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cb.release();
        return hip_fail(ctx, e, "copy");
    }
    ctx->cam.release();
    ctx->cam = cb;
    ctx->cams = cams;
    ctx->V = V;
    ctx->H = H;
    ctx->W = W;
    return ART_OK;
}

art_status art_render(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                      float lambda_th, unsigned flags, float* out_feat, float* out_alpha,
                      float* out_tfinal) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_alpha) return fail(ctx, ART_EINVAL, "out_feat / out_alpha is NULL");
    DeviceGuard g(ctx->device);
    PassOut o;
    o.out_feat = out_feat;
    o.out_alpha = out_alpha;
    o.out_tfinal = out_tfinal;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags, 0, o, 0, ctx->P);
}

art_status art_backward(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                        float lambda_th, unsigned flags, const float* out_feat, const float* out_tfinal,
                        const float* d_feat, const float* d_alpha, float* d_sigma, float* d_leaf_feat) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_tfinal || !d_feat || !d_sigma || !d_leaf_feat)
        return fail(ctx, ART_EINVAL, "backward needs out_feat, out_tfinal, d_feat, d_sigma, d_leaf_feat");
    DeviceGuard g(ctx->device);
    PassOut o;
    o.fwd_feat = out_feat;
    o.fwd_tfinal = out_tfinal;
    o.d_feat = d_feat;
    o.d_alpha = d_alpha;
    o.d_sigma = d_sigma;
    o.d_leaf_feat = d_leaf_feat;
    o.reuse = (flags & ART_REUSE_BUILD) != 0;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags & ~ART_REUSE_BUILD, 1, o, 0, ctx->P);
}

// Ray checkpoints: K records of C + 4 words per ray, one every `every` samples.
static art_status check_ckpt(art_ctx* ctx, int K, int every, const float* ckpt, const int32_t* ckpt_n) {
    if (!ckpt || !ckpt_n) return fail(ctx, ART_EINVAL, "ckpt / ckpt_n is NULL");
    if (K < 1 || K > 64) return fail(ctx, ART_EINVAL, "K must be in 1..64");
    if (every < 1 || every > 65536) return fail(ctx, ART_EINVAL, "every must be in 1..65536");
    if ((reinterpret_cast<uintptr_t>(ckpt) & 7u) != 0) return fail(ctx, ART_EINVAL, "ckpt must be 8-byte aligned");
    return ART_OK;
}

art_status art_render_ckpt(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                           float lambda_th, unsigned flags, float* out_feat, float* out_alpha, float* out_tfinal,
                           int K, int every, float* ckpt, int32_t* ckpt_n) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_alpha || !out_tfinal) return fail(ctx, ART_EINVAL, "out_feat / out_alpha / out_tfinal is NULL");
    art_status rc = check_ckpt(ctx, K, every, ckpt, ckpt_n);
    if (rc != ART_OK) return rc;
    DeviceGuard g(ctx->device);
    PassOut o;
    o.out_feat = out_feat;
    o.out_alpha = out_alpha;
    o.out_tfinal = out_tfinal;
    o.ckpt = ckpt;
    o.ckpt_n = ckpt_n;
    o.ckpt_K = K;
    o.ckpt_every = every;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags, 7, o, 0, ctx->P);
}

art_status art_backward_ckpt(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                             float lambda_th, unsigned flags, const float* out_feat, const float* out_tfinal,
                             const float* d_feat, const float* d_alpha, float* d_sigma, float* d_leaf_feat, int K,
                             int every, const float* ckpt, const int32_t* ckpt_n) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_tfinal || !d_feat || !d_sigma || !d_leaf_feat)
        return fail(ctx, ART_EINVAL, "backward needs out_feat, out_tfinal, d_feat, d_sigma, d_leaf_feat");
    art_status rc = check_ckpt(ctx, K, every, ckpt, ckpt_n);
    if (rc != ART_OK) return rc;
    DeviceGuard g(ctx->device);
    PassOut o;
    o.fwd_feat = out_feat;
    o.fwd_tfinal = out_tfinal;
    o.d_feat = d_feat;
    o.d_alpha = d_alpha;
    o.d_sigma = d_sigma;
    o.d_leaf_feat = d_leaf_feat;
    o.reuse = (flags & ART_REUSE_BUILD) != 0;
    o.ckpt = const_cast<float*>(ckpt);   // read only in the adjoint
    o.ckpt_n = const_cast<int32_t*>(ckpt_n);
    o.ckpt_K = K;
    o.ckpt_every = every;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags & ~ART_REUSE_BUILD, 1, o, 0, ctx->P);
}

art_status art_render_depth(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                            float lambda_th, unsigned flags, float depth_sigma, float* out_feat, float* out_alpha,
                            float* out_tfinal, float* out_depth) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_alpha || !out_depth) return fail(ctx, ART_EINVAL, "out_feat / out_alpha / out_depth is NULL");
    if (!(depth_sigma == depth_sigma)) return fail(ctx, ART_EINVAL, "depth_sigma is NaN");
    DeviceGuard g(ctx->device);
    PassOut o;
    o.out_feat = out_feat;
    o.out_alpha = out_alpha;
    o.out_tfinal = out_tfinal;
    o.out_depth = out_depth;
    o.depth_sigma = depth_sigma;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags, 5, o, 0, ctx->P);
}

art_status art_render_sh(art_ctx* ctx, int C, int H, art_dtype dtype, const void* sigma, const void* feat,
                         float lambda_th, unsigned flags, float* out_feat, float* out_alpha, float* out_tfinal) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_alpha) return fail(ctx, ART_EINVAL, "out_feat / out_alpha is NULL");
    if (H != 1 && H != 4 && H != 9) return fail(ctx, ART_EUNSUPPORTED, "H must be 1, 4 or 9 (SH degree <= 2)");
    if (ctx->J > kMaxBonesSH)
        return fail(ctx, ART_EUNSUPPORTED, "view-dependent features support at most " + std::to_string(kMaxBonesSH) +
                                               " bones");
    DeviceGuard g(ctx->device);
    PassOut o;
    o.out_feat = out_feat;
    o.out_alpha = out_alpha;
    o.out_tfinal = out_tfinal;
    o.sh_H = H;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags, 6, o, 0, ctx->P);
}

int64_t art_shading_param_count(int C) {
    if (C < 1 || C > 32) return -1;
    int64_t n = 0;
    for (int l = 0; l < kShadeLayers; ++l) n += (int64_t)kShade[l].cout * shade_cin(l, C) * 9 + kShade[l].cout;
    return n + 4 * 32 + 4;
}

art_status art_shading_set_weights(art_ctx* ctx, int C, int64_t count, const float* w) {
    if (!ctx) return ART_EINVAL;
    if (C < 1 || C > 32) return fail(ctx, ART_EUNSUPPORTED, "C must be in 1..32");
    if (!w || count != art_shading_param_count(C)) return fail(ctx, ART_EINVAL, "weight count mismatch or NULL");
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(w[i])) return fail(ctx, ART_EINVAL, "weights must be finite");
    // PyTorch layout [Cout][Cin][3][3] + bias per layer -> FP16 [3][3][Cout][Cin_pad] + FP32 bias
    std::vector<_Float16> hw;
    std::vector<float> hb, hh(4 * 32 + 4);
    const float* p = w;
    for (int l = 0; l < kShadeLayers; ++l) {
        const int co = kShade[l].cout, ci = shade_cin(l, C), cp = shade_cin_pad(l);
        const size_t base = hw.size();
        hw.resize(base + (size_t)9 * co * cp, (_Float16)0.0f);
        for (int o = 0; o < co; ++o)
            for (int i = 0; i < ci; ++i)
                for (int k = 0; k < 9; ++k) hw[base + ((size_t)k * co + o) * cp + i] = (_Float16)p[((size_t)o * ci + i) * 9 + k];
        p += (size_t)co * ci * 9;
        hb.insert(hb.end(), p, p + co);
        p += co;
    }
    std::copy(p, p + 4 * 32 + 4, hh.begin());
    DeviceGuard g(ctx->device);
    ART_TRY_HIP(ctx->shade_w.ensure(hw.size() * 2), "device allocation");
    ART_TRY_HIP(ctx->shade_b.ensure(hb.size() * 4), "device allocation");
    ART_TRY_HIP(ctx->shade_head.ensure(hh.size() * 4), "device allocation");
    ART_TRY_HIP(hipMemcpy(ctx->shade_w.p, hw.data(), hw.size() * 2, hipMemcpyHostToDevice), "copy");
    ART_TRY_HIP(hipMemcpy(ctx->shade_b.p, hb.data(), hb.size() * 4, hipMemcpyHostToDevice), "copy");
    ART_TRY_HIP(hipMemcpy(ctx->shade_head.p, hh.data(), hh.size() * 4, hipMemcpyHostToDevice), "copy");
    ctx->shade_C = C;
    return ART_OK;
}

}  // extern "C"

namespace {
art_status shade_check(art_ctx* ctx, int C, int N, int H, int W, const float* F, const float* out) {
    if (ctx->shade_C == 0 || ctx->shade_C != C) return fail(ctx, ART_ESTATE, "no shading weights for this C");
    if (N < 1 || H < 8 || W < 8 || (H % 8) || (W % 8)) return fail(ctx, ART_EINVAL, "N >= 1; H, W multiples of 8");
    if (!F || !out) return fail(ctx, ART_EINVAL, "F / out is NULL");
    return ART_OK;
}

// The network on N maps with its activations at `base` (laid out by shade_layout).
art_status shade_run(art_ctx* ctx, int C, int N, int H, int W, const float* F, float* out, uint16_t* base,
                     const size_t off[kShadeBufs]) {
    hipStream_t st = ctx->stream;
    uint16_t* X = base + off[0];
    uint16_t* T0 = base + off[1];
    uint16_t* E0 = base + off[2];
    uint16_t* P0 = base + off[3];
    uint16_t* T1 = base + off[4];
    uint16_t* E1 = base + off[5];
    uint16_t* P1 = base + off[6];
    uint16_t* T2 = base + off[7];
    uint16_t* E2 = base + off[8];
    uint16_t* P2 = base + off[9];
    uint16_t* T3 = base + off[10];
    uint16_t* Bt = base + off[11];
    const uint16_t* wl[kShadeLayers];
    const float* bl[kShadeLayers];
    {
        const uint16_t* wp = ctx->shade_w.as<uint16_t>();
        const float* bp = ctx->shade_b.as<float>();
        for (int l = 0; l < kShadeLayers; ++l) {
            wl[l] = wp;
            bl[l] = bp;
            wp += (size_t)9 * kShade[l].cout * shade_cin_pad(l);
            bp += kShade[l].cout;
        }
    }
    auto conv = [&](int l, const uint16_t* s1, int c1, const uint16_t* s2, int c2, uint16_t* o, int h, int w,
                    float* head_out = nullptr) {
        ConvLaunch a{};
        a.src1 = s1;
        a.C1 = c1;
        a.src2 = s2;
        a.C2 = c2;
        a.wgt = wl[l];
        a.bias = bl[l];
        a.out = o;
        a.N = N;
        a.H = h;
        a.W = w;
        a.Cout = kShade[l].cout;
        a.relu = 1;
        if (head_out) {
            const ConvHead hd{ctx->shade_head.as<float>(), ctx->shade_head.as<float>() + 128, head_out};
            return launch_conv3x3_head(a, hd, st);
        }
        return launch_conv3x3(a, st);
    };
    hipError_t e = launch_to_nhwc(F, N, C, H, W, 32, X, st);
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    if (e == hipSuccess) e = conv(0, X, 32, nullptr, 0, T0, H, W);
    if (e == hipSuccess) e = conv(1, T0, 32, nullptr, 0, E0, H, W);
    if (e == hipSuccess) e = launch_maxpool2(E0, N, H, W, 32, P0, st);
    if (e == hipSuccess) e = conv(2, P0, 32, nullptr, 0, T1, H1, W1);
    if (e == hipSuccess) e = conv(3, T1, 64, nullptr, 0, E1, H1, W1);
    if (e == hipSuccess) e = launch_maxpool2(E1, N, H1, W1, 64, P1, st);
    if (e == hipSuccess) e = conv(4, P1, 64, nullptr, 0, T2, H2, W2);
    if (e == hipSuccess) e = conv(5, T2, 128, nullptr, 0, E2, H2, W2);
    if (e == hipSuccess) e = launch_maxpool2(E2, N, H2, W2, 128, P2, st);
    if (e == hipSuccess) e = conv(6, P2, 128, nullptr, 0, T3, H3, W3);
    if (e == hipSuccess) e = conv(7, T3, 256, nullptr, 0, Bt, H3, W3);
    if (e == hipSuccess) e = conv(8, E2, 128, Bt, 256, T2, H2, W2);
    if (e == hipSuccess) e = conv(9, T2, 128, nullptr, 0, E2, H2, W2);
    if (e == hipSuccess) e = conv(10, E1, 64, E2, 128, T1, H1, W1);
    if (e == hipSuccess) e = conv(11, T1, 64, nullptr, 0, E1, H1, W1);
    if (e == hipSuccess) e = conv(12, E0, 32, E1, 64, T0, H, W);
    if (fused_shading_head()) {   // the last convolution writes the head's sigmoid outputs
        if (e == hipSuccess) e = conv(13, T0, 32, nullptr, 0, nullptr, H, W, out);
    } else {
        if (e == hipSuccess) e = conv(13, T0, 32, nullptr, 0, X, H, W);
        if (e == hipSuccess)
            e = launch_head(X, N, H, W, ctx->shade_head.as<float>(), ctx->shade_head.as<float>() + 128, out, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "shading network");
    return ART_OK;
}

}  // namespace

extern "C" {

art_status art_shading_forward(art_ctx* ctx, int C, int N, int H, int W, const float* F, float* out) {
    if (!ctx) return ART_EINVAL;
    art_status rc = shade_check(ctx, C, N, H, W, F, out);
    if (rc != ART_OK) return rc;
    DeviceGuard g(ctx->device);
    size_t off[kShadeBufs];
    const size_t tot = shade_layout((size_t)N * H * W, off);
    rc = ensure_bufs(ctx, {{&ctx->shade_act, tot * 2}});
    if (rc != ART_OK) return rc;
    return shade_run(ctx, C, N, H, W, F, out, ctx->shade_act.as<uint16_t>(), off);
}

art_status art_shading_forward_noalloc(art_ctx* ctx, int C, int N, int H, int W, const float* F, float* out) {
    if (!ctx) return ART_EINVAL;
    art_status rc = shade_check(ctx, C, N, H, W, F, out);
    if (rc != ART_OK) return rc;
    size_t off[kShadeBufs];
    const size_t tot = shade_layout((size_t)N * H * W, off);
    if (tot * 2 > (size_t)ART_SHADING_NOALLOC_BYTES)
        return fail(ctx, ART_EINVAL, "the batch needs " + std::to_string(tot * 2) +
                                         " bytes of activations, above the fixed array of " +
                                         std::to_string((size_t)ART_SHADING_NOALLOC_BYTES) + " bytes");
    if (!ctx->shade_fixed) return fail(ctx, ART_EDEVICE, "fixed activation array not resolved");
    DeviceGuard g(ctx->device);
    return shade_run(ctx, C, N, H, W, F, out, static_cast<uint16_t*>(ctx->shade_fixed), off);
}

art_status art_vrt(art_ctx* ctx, int C, art_dtype dtype, const void* feat, float lambda_vrt, unsigned flags,
                   float* d_feat, double* loss) {
    if (!ctx) return ART_EINVAL;
    if (!feat || !d_feat || !loss) return fail(ctx, ART_EINVAL, "feat / d_feat / loss is NULL");
    if (!(lambda_vrt >= 0.0f && lambda_vrt < 1e30f)) return fail(ctx, ART_EINVAL, "lambda_vrt must be finite and >= 0");
    if (!supported_C(C)) return fail(ctx, ART_EUNSUPPORTED, "C must be 4, 8, 16 or 32");
    if (dtype != ART_F32 && dtype != ART_BF16) return fail(ctx, ART_EINVAL, "dtype must be ART_F32 or ART_BF16");
    if (flags & ~(ART_GEOM_FP32 | ART_REUSE_BUILD)) return fail(ctx, ART_EINVAL, "unknown flag bits");
    art_status rc = check_build_state(ctx);
    if (rc != ART_OK) return rc;
    DeviceGuard g(ctx->device);
    CallPlan pl;   // octrees only: no cameras involved
    pl.C = C;
    pl.storage = dtype == ART_BF16 ? 1 : 0;
    pl.fp32 = (flags & ART_GEOM_FP32) != 0;
    pl.Vg = 1;
    pl.ngroups = 1;
    if (ctx->s.pair_cap == 0) ctx->s.pair_cap = initial_pair_cap(1);
    const int slots = (int)std::min<size_t>((size_t)ctx->P,
                                            std::max<size_t>(1, slot_budget_bytes(ctx) / slot_bytes(ctx, pl, ctx->s.pair_cap)));
    rc = ensure_scratch(ctx, pl, slots);
    if (rc != ART_OK) return rc;
    hipStream_t st = ctx->stream;
    Scratch& s = ctx->s;
    int launches = 0;
    Timing tm;
    ART_TRY_HIP(launch_fill_u32(s.stats.as<uint32_t>(), 0u, 32, st), "fill");
    ART_TRY_HIP(launch_fill_u32(s.loss.as<uint32_t>(), 0u, 2, st), "fill");
    // the octrees of a whole-batch render (any view grouping: only the octrees are read)
    const art_ctx::BuildMemo& m = ctx->memo;
    if ((flags & ART_REUSE_BUILD) && m.valid && m.version == ctx->state_version && m.fp32 == pl.fp32 &&
        m.P == ctx->P && m.occ == s.occ_win.p && m.rows == s.keys1.p && m.counters == s.counters.p) {
        ART_TRY_HIP(launch_vrt(s.keys1.as<uint32_t>(), s.occ_win.as<uint32_t>(), (uint32_t)ctx->n, C, pl.storage, feat,
                               s.counters.as<PoseCounters>(), lambda_vrt, ctx->P, d_feat, s.loss.as<double>(), st),
                    "vrt");
    } else {
    ART_TRY_HIP(launch_fk(ctx->parent.as<int32_t>(), ctx->rest.as<double>(), ctx->pose.as<double>(), ctx->J,
                          ctx->P, ctx->Gtmp.as<double>(), ctx->B64.as<double>(), ctx->B32.as<float>(), st),
                "fk");
    for (int p0 = 0; p0 < ctx->P; p0 += slots) {
        const int batch = std::min(ctx->P, p0 + slots) - p0;
        rc = build_batch(ctx, pl, p0, batch, nullptr, feat, &launches, tm);
        if (rc != ART_OK) return rc;
        ART_TRY_HIP(launch_vrt(s.keys1.as<uint32_t>(), s.occ_win.as<uint32_t>(), (uint32_t)ctx->n, C, pl.storage,
                               feat, s.counters.as<PoseCounters>(), lambda_vrt, batch, d_feat, s.loss.as<double>(), st),
                    "vrt");
    }
    }
    double h = 0.0;
    ART_TRY_HIP(hipMemcpyAsync(&h, s.loss.p, 8, hipMemcpyDeviceToHost, st), "copy");
    ART_TRY_HIP(hipStreamSynchronize(st), "vrt");
    *loss = h;
    return ART_OK;
}

art_status art_query(art_ctx* ctx, int pose, unsigned flags, int64_t n, const double* points, int32_t* leaf) {
    if (!ctx) return ART_EINVAL;
    if (n < 0) return fail(ctx, ART_EINVAL, "n must be >= 0");
    if (n > 0 && (!points || !leaf)) return fail(ctx, ART_EINVAL, "points / leaf is NULL");
    if (flags & ~ART_GEOM_FP32) return fail(ctx, ART_EINVAL, "unknown flag bits");
    art_status rc = check_build_state(ctx);
    if (rc != ART_OK) return rc;
    if (pose < 0 || pose >= ctx->P) return fail(ctx, ART_EINVAL, "pose out of range");
    DeviceGuard g(ctx->device);
    CallPlan pl;
    pl.C = 4;
    pl.storage = 0;
    pl.fp32 = (flags & ART_GEOM_FP32) != 0;
    pl.Vg = 1;
    pl.ngroups = 1;
    if (ctx->s.pair_cap == 0) ctx->s.pair_cap = initial_pair_cap(1);
    rc = ensure_scratch(ctx, pl, 1);
    if (rc != ART_OK) return rc;
    hipStream_t st = ctx->stream;
    Timing tm;
    int launches = 0;
    ART_TRY_HIP(launch_fill_u32(ctx->s.stats.as<uint32_t>(), 0u, 32, st), "fill");
    ART_TRY_HIP(launch_fk(ctx->parent.as<int32_t>(), ctx->rest.as<double>(), ctx->pose.as<double>(), ctx->J,
                          ctx->P, ctx->Gtmp.as<double>(), ctx->B64.as<double>(), ctx->B32.as<float>(), st),
                "fk");
    rc = build_batch(ctx, pl, pose, 1, nullptr, nullptr, &launches, tm);
    if (rc != ART_OK) return rc;
    ART_TRY_HIP(launch_query(points, n, ctx->depth, octree_slot(ctx, pl, 0), ctx->s.counters.as<PoseCounters>(),
                             leaf, st),
                "query");
    ART_TRY_HIP(hipStreamSynchronize(st), "query");
    return ART_OK;
}

art_status art_flut_adam(art_ctx* ctx, int64_t count, float* param, const float* grad, float* m, float* v, int step,
                         float lr, float beta1, float beta2, float eps, float lower) {
    if (!ctx) return ART_EINVAL;
    if (count < 0) return fail(ctx, ART_EINVAL, "count must be >= 0");
    if (count > 0 && (!param || !grad || !m || !v)) return fail(ctx, ART_EINVAL, "NULL buffer");
    if (step < 1) return fail(ctx, ART_EINVAL, "step counts from 1");
    if (!(lr >= 0.0f && lr < 1e30f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f && eps < 1e30f) || lower != lower)
        return fail(ctx, ART_EINVAL, "invalid Adam parameters");
    DeviceGuard g(ctx->device);
    AdamStep a;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    a.bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    ART_TRY_HIP(launch_flut_adam(param, grad, m, v, count, a, lower, ctx->stream), "flut adam");
    return ART_OK;
}

art_status art_proposal_labels(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                               float lambda_th, unsigned flags, float* labels) {
    if (!ctx) return ART_EINVAL;
    if (!labels) return fail(ctx, ART_EINVAL, "labels is NULL");
    DeviceGuard g(ctx->device);
    PassOut o;
    o.labels = labels;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags, 3, o, 0, ctx->P);
}

art_status art_render_proposal(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                               float lambda_th, unsigned flags, const float* intervals, float margin_h,
                               float f2_tau, float* out_feat, float* out_alpha, float* out_tfinal) {
    if (!ctx) return ART_EINVAL;
    if (!out_feat || !out_alpha) return fail(ctx, ART_EINVAL, "out_feat / out_alpha is NULL");
    if (!(margin_h >= 0.0f && margin_h < 1e30f)) return fail(ctx, ART_EINVAL, "margin_h must be finite and >= 0");
    if (!(f2_tau == f2_tau)) return fail(ctx, ART_EINVAL, "f2_tau is NaN");
    DeviceGuard g(ctx->device);
    if (!intervals) {
        art_status rc = check_render_state(ctx);
        if (rc != ART_OK) return rc;
        rc = mlp_prepare(ctx);
        if (rc != ART_OK) return rc;
    }
    PassOut o;
    o.out_feat = out_feat;
    o.out_alpha = out_alpha;
    o.out_tfinal = out_tfinal;
    o.intervals = intervals;
    o.margin = (float)(margin_h / (double)(1 << std::max(ctx->depth, 0)));
    o.f2_tau = f2_tau;
    o.near_only = (flags & ART_PROPOSAL_NEAR_ONLY) != 0;
    return render_call(ctx, C, dtype, sigma, feat, lambda_th, flags & ~ART_PROPOSAL_NEAR_ONLY, 4, o, 0, ctx->P);
}

int64_t art_proposal_param_count(int J) {
    if (J < 1 || J > 255) return -1;
    return mlp_dims(J).np;
}

art_status art_proposal_set_weights(art_ctx* ctx, int64_t count, const float* w) {
    if (!ctx) return ART_EINVAL;
    if (ctx->J <= 0) return fail(ctx, ART_ESTATE, "no skeleton (art_set_skeleton)");
    const MlpDims m = mlp_dims(ctx->J);
    if (!w || count != m.np)
        return fail(ctx, ART_EINVAL, "expected " + std::to_string(m.np) + " weights for J = " + std::to_string(ctx->J));
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(w[i])) return fail(ctx, ART_EINVAL, "weights must be finite");
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    const size_t bytes = (size_t)m.np * 4;
    art_status rc = ensure_bufs(ctx, {{&ctx->mlp_theta, bytes}, {&ctx->mlp_m1, bytes}, {&ctx->mlp_m2, bytes}});
    if (rc != ART_OK) return rc;
    ART_TRY_HIP(hipMemcpyAsync(ctx->mlp_theta.p, w, bytes, hipMemcpyHostToDevice, st), "copy");
    ART_TRY_HIP(launch_fill_u32(ctx->mlp_m1.as<uint32_t>(), 0u, (size_t)m.np, st), "fill");
    ART_TRY_HIP(launch_fill_u32(ctx->mlp_m2.as<uint32_t>(), 0u, (size_t)m.np, st), "fill");
    ART_TRY_HIP(hipStreamSynchronize(st), "copy");
    ctx->mlp_J = ctx->J;
    ctx->mlp_step = 0;
    return ART_OK;
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output k (k = 1, 2, ...) of the stream of `seed`.
static uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

art_status art_proposal_init(art_ctx* ctx, uint64_t seed) {
    if (!ctx) return ART_EINVAL;
    if (ctx->J <= 0) return fail(ctx, ART_ESTATE, "no skeleton (art_set_skeleton)");
    const MlpDims m = mlp_dims(ctx->J);
    // parameter i (flat order) takes output i + 1 of the stream: its top 24
    // bits give u in [0, 1), the value (2u - 1) / sqrt(fan-in of its layer)
    const int fan_in[4] = {m.n_in, 64, 64, 64};
    const int start[5] = {m.oW1, m.oW2, m.oW3, m.oW4, m.np};
    std::vector<float> w((size_t)m.np);
    for (int l = 0; l < 4; ++l) {
        const double k = 1.0 / std::sqrt((double)fan_in[l]);
        for (int i = start[l]; i < start[l + 1]; ++i) {
            const double u = (double)(splitmix64(seed, (uint64_t)i + 1u) >> 40) * 0x1.0p-24;
            w[(size_t)i] = (float)((2.0 * u - 1.0) * k);
        }
    }
    return art_proposal_set_weights(ctx, m.np, w.data());
}

art_status art_proposal_get_weights(art_ctx* ctx, int64_t count, float* w) {
    if (!ctx) return ART_EINVAL;
    if (ctx->mlp_J <= 0 || ctx->mlp_J != ctx->J)
        return fail(ctx, ART_ESTATE, "no proposal weights for the current skeleton (art_proposal_set_weights)");
    const MlpDims m = mlp_dims(ctx->J);
    if (!w || count != m.np) return fail(ctx, ART_EINVAL, "expected " + std::to_string(m.np) + " weights");
    DeviceGuard g(ctx->device);
    ART_TRY_HIP(hipMemcpyAsync(w, ctx->mlp_theta.p, (size_t)m.np * 4, hipMemcpyDeviceToHost, ctx->stream), "copy");
    ART_TRY_HIP(hipStreamSynchronize(ctx->stream), "copy");
    return ART_OK;
}

art_status art_proposal_gather(art_ctx* ctx, int64_t n, const int64_t* ray_id, const float* labels, float* od,
                               int32_t* pose, float* target) {
    if (!ctx) return ART_EINVAL;
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    if (ctx->V <= 0) return fail(ctx, ART_ESTATE, "no cameras (art_set_cameras)");
    if (n < 0) return fail(ctx, ART_EINVAL, "n must be >= 0");
    if (n > 0 && (!ray_id || !labels || !od || !pose || !target)) return fail(ctx, ART_EINVAL, "NULL buffer");
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    {
        const art_status rf = ensure_bufs(ctx, {{&ctx->mlp_flag, 64}});
        if (rf != ART_OK) return rf;
    }
    ART_TRY_HIP(launch_fill_u32(ctx->mlp_flag.as<uint32_t>(), 0u, 1, st), "fill");
    ART_TRY_HIP(launch_mlp_gather(ray_id, n, labels, ctx->cam.as<CamParams>(), ctx->P, ctx->V, ctx->H, ctx->W, od,
                                  pose, target, ctx->mlp_flag.as<uint32_t>(), st),
                "gather");
    uint32_t bad = 0;
    ART_TRY_HIP(hipMemcpyAsync(&bad, ctx->mlp_flag.p, 4, hipMemcpyDeviceToHost, st), "copy");
    ART_TRY_HIP(hipStreamSynchronize(st), "gather");
    if (bad) return fail(ctx, ART_EINVAL, "ray id outside [0, P*V*H*W)");
    return ART_OK;
}

namespace {
constexpr int64_t kMaxMlpBatch = (int64_t)1 << 20;

art_status check_bad_pose(art_ctx* ctx) {
    uint32_t bad = 0;
    ART_TRY_HIP(hipMemcpyAsync(&bad, ctx->mlp_flag.p, 4, hipMemcpyDeviceToHost, ctx->stream), "copy");
    ART_TRY_HIP(hipStreamSynchronize(ctx->stream), "proposal network");
    if (bad) return fail(ctx, ART_EINVAL, "pose id outside [0, P)");
    return ART_OK;
}

art_status ensure_mlp_train_bufs(art_ctx* ctx, int64_t n) {
    const MlpDims m = mlp_dims(ctx->J);
    const size_t chunks = (size_t)(mlp_pad(n) / 256);
    return ensure_bufs(ctx, {{&ctx->mlp_S, mlp_scratch_bytes(n)},
                             {&ctx->mlp_part, chunks * (size_t)m.np * 4},
                             {&ctx->mlp_lossp, (size_t)mlp_loss_parts(n) * 4},
                             {&ctx->mlp_flag, 64}});
}
}  // namespace

art_status art_proposal_forward(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, float* out) {
    if (!ctx) return ART_EINVAL;
    if (n < 0) return fail(ctx, ART_EINVAL, "n must be >= 0");
    if (n > 0 && (!od || !pose || !out)) return fail(ctx, ART_EINVAL, "NULL buffer");
    DeviceGuard g(ctx->device);
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    art_status rc = mlp_prepare(ctx);
    if (rc != ART_OK) return rc;
    if (n == 0) return ART_OK;
    {
        const art_status rf = ensure_bufs(ctx, {{&ctx->mlp_flag, 64}});
        if (rf != ART_OK) return rf;
    }
    ART_TRY_HIP(launch_fill_u32(ctx->mlp_flag.as<uint32_t>(), 0u, 1, ctx->stream), "fill");
    ART_TRY_HIP(launch_mlp_forward(ctx->mlp_packed.as<uint16_t>(), ctx->mlp_theta.as<float>(),
                                   ctx->mlp_cbias.as<float>(), mlp_dims(ctx->J), od, pose, ctx->P, n, out,
                                   ctx->mlp_flag.as<uint32_t>(), ctx->stream),
                "proposal forward");
    return check_bad_pose(ctx);
}

art_status art_proposal_set_loss(art_ctx* ctx, int kind, float tau_near, float tau_far) {
    if (!ctx) return ART_EINVAL;
    if (kind != 0 && kind != 1) return fail(ctx, ART_EINVAL, "loss kind must be 0 (SmoothL1) or 1 (pinball)");
    if (kind == 1 && !(tau_near > 0.0f && tau_near < 1.0f && tau_far > 0.0f && tau_far < 1.0f))
        return fail(ctx, ART_EINVAL, "pinball levels must be in (0, 1)");
    ctx->mlp_loss_fn.kind = kind;
    ctx->mlp_loss_fn.tau[0] = kind == 1 ? tau_near : 0.5f;
    ctx->mlp_loss_fn.tau[1] = kind == 1 ? tau_far : 0.5f;
    return ART_OK;
}

art_status art_proposal_grad(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, const float* target,
                             float* grad, float* loss) {
    if (!ctx) return ART_EINVAL;
    if (n < 1 || n > kMaxMlpBatch) return fail(ctx, ART_EINVAL, "n must be in 1..2^20");
    if (!od || !pose || !target || !grad || !loss) return fail(ctx, ART_EINVAL, "NULL buffer");
    DeviceGuard g(ctx->device);
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    art_status rc = mlp_prepare(ctx);
    if (rc != ART_OK) return rc;
    rc = ensure_mlp_train_bufs(ctx, n);
    if (rc != ART_OK) return rc;
    hipStream_t st = ctx->stream;
    const MlpDims m = mlp_dims(ctx->J);
    ART_TRY_HIP(launch_fill_u32(ctx->mlp_flag.as<uint32_t>(), 0u, 1, st), "fill");
    ART_TRY_HIP(launch_mlp_grad(ctx->mlp_packed.as<uint16_t>(), ctx->mlp_theta.as<float>(), ctx->mlp_cbias.as<float>(),
                                ctx->mlp_code.as<float>(), m, od, pose, target, ctx->P, n, ctx->mlp_S.as<float>(),
                                ctx->mlp_part.as<float>(), ctx->mlp_lossp.as<float>(), ctx->mlp_flag.as<uint32_t>(),
                                ctx->mlp_loss_fn, st),
                "proposal gradient");
    ART_TRY_HIP(launch_mlp_reduce(ctx->mlp_part.as<float>(), n, m, grad, ctx->mlp_theta.as<float>(), nullptr, nullptr,
                                  nullptr, ctx->mlp_lossp.as<float>(), loss, st),
                "proposal gradient");
    return check_bad_pose(ctx);
}

art_status art_proposal_train(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, const float* target,
                              int64_t batch, int steps, float lr, float beta1, float beta2, float eps,
                              float* loss_log) {
    if (!ctx) return ART_EINVAL;
    if (batch < 1 || batch > kMaxMlpBatch) return fail(ctx, ART_EINVAL, "batch must be in 1..2^20");
    if (n < batch) return fail(ctx, ART_EINVAL, "n must be >= batch");
    if (steps < 0) return fail(ctx, ART_EINVAL, "steps must be >= 0");
    if (!(lr > 0.0f && lr < 1e30f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f && eps < 1e30f))
        return fail(ctx, ART_EINVAL, "Adam hyper-parameters out of range");
    if (!od || !pose || !target) return fail(ctx, ART_EINVAL, "NULL buffer");
    DeviceGuard g(ctx->device);
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    art_status rc = mlp_prepare(ctx);
    if (rc != ART_OK) return rc;
    rc = ensure_mlp_train_bufs(ctx, batch);
    if (rc != ART_OK) return rc;
    rc = ensure_bufs(ctx, {{&ctx->mlp_loss, (size_t)std::max(steps, 1) * 4}});
    if (rc != ART_OK) return rc;
    hipStream_t st = ctx->stream;
    const MlpDims m = mlp_dims(ctx->J);
    const int64_t nb = n / batch;
    ART_TRY_HIP(launch_fill_u32(ctx->mlp_flag.as<uint32_t>(), 0u, 1, st), "fill");
    for (int s = 0; s < steps; ++s) {
        const int64_t off = (s % nb) * batch;
        if (s > 0)   // operands and pose biases of the updated weights
            ART_TRY_HIP(launch_mlp_prep(ctx->mlp_theta.as<float>(), m, ctx->mlp_code.as<float>(), ctx->P,
                                        ctx->mlp_packed.as<uint16_t>(), ctx->mlp_cbias.as<float>(), st),
                        "proposal prep");
        ART_TRY_HIP(launch_mlp_grad(ctx->mlp_packed.as<uint16_t>(), ctx->mlp_theta.as<float>(),
                                    ctx->mlp_cbias.as<float>(), ctx->mlp_code.as<float>(), m, od + off * 6,
                                    pose + off, target + off * 2, ctx->P, batch, ctx->mlp_S.as<float>(),
                                    ctx->mlp_part.as<float>(), ctx->mlp_lossp.as<float>(),
                                    ctx->mlp_flag.as<uint32_t>(), ctx->mlp_loss_fn, st),
                    "proposal gradient");
        const int64_t t = ++ctx->mlp_step;
        AdamStep ad;
        ad.lr = lr;
        ad.beta1 = beta1;
        ad.beta2 = beta2;
        ad.eps = eps;
        ad.bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
        ad.bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
        ART_TRY_HIP(launch_mlp_reduce(ctx->mlp_part.as<float>(), batch, m, nullptr, ctx->mlp_theta.as<float>(),
                                      ctx->mlp_m1.as<float>(), ctx->mlp_m2.as<float>(), &ad, ctx->mlp_lossp.as<float>(),
                                      ctx->mlp_loss.as<float>() + s, st),
                    "proposal Adam step");
    }
    if (loss_log && steps > 0)
        ART_TRY_HIP(hipMemcpyAsync(loss_log, ctx->mlp_loss.p, (size_t)steps * 4, hipMemcpyDeviceToHost, st), "copy");
    return check_bad_pose(ctx);
}

art_status art_get_hits(art_ctx* ctx, int pose, int view, int C, art_dtype dtype, const void* sigma,
                        const void* feat, float lambda_th, unsigned flags, int max_hits, int32_t* leaf,
                        double* delta, int32_t* count) {
    if (!ctx) return ART_EINVAL;
    if (pose < 0 || pose >= ctx->P || view < 0 || view >= ctx->V)
        return fail(ctx, ART_EINVAL, "pose / view out of range");
    if (max_hits < 1 || !leaf || !delta || !count) return fail(ctx, ART_EINVAL, "hit buffers");
    if (!supported_C(C)) return fail(ctx, ART_EUNSUPPORTED, "C must be 4, 8, 16 or 32");
    DeviceGuard g(ctx->device);
    const size_t HW = (size_t)ctx->H * ctx->W;
    DevBuf tf, ta;   // forward maps of the pose's views, discarded
    ART_TRY_HIP(tf.ensure(HW * C * 4 * ctx->V), "device allocation");
    hipError_t e = ta.ensure(HW * 4 * ctx->V);
    if (e != hipSuccess) {
        tf.release();
        return hip_fail(ctx, e, "device allocation");
    }
    PassOut o;
    o.single_pose = true;
    o.out_feat = tf.as<float>();
    o.out_alpha = ta.as<float>();
    o.max_hits = max_hits;
    o.debug_view = view;
    o.hit_leaf = leaf;
    o.hit_delta = delta;
    o.hit_count = count;
    // the hit lists are complete when the call returns (ART_ASYNC does not apply)
    art_status rc = render_call(ctx, C, dtype, sigma, feat, lambda_th, flags & ~ART_ASYNC, 2, o, pose, pose + 1);
    tf.release();
    ta.release();
    return rc;
}

art_status art_get_bones(art_ctx* ctx, double* B) {
    if (!ctx) return ART_EINVAL;
    if (!B) return fail(ctx, ART_EINVAL, "B is NULL");
    if (ctx->J <= 0) return fail(ctx, ART_ESTATE, "no skeleton (art_set_skeleton)");
    if (ctx->P <= 0) return fail(ctx, ART_ESTATE, "no poses (art_set_poses)");
    DeviceGuard g(ctx->device);
    const size_t nb = (size_t)ctx->P * ctx->J * 12;
    {
        const art_status rb = ensure_bufs(ctx, {{&ctx->B64, nb * 8}, {&ctx->B32, nb * 4}, {&ctx->Gtmp, nb * 8}});
        if (rb != ART_OK) return rb;
    }
    ART_TRY_HIP(launch_fk(ctx->parent.as<int32_t>(), ctx->rest.as<double>(), ctx->pose.as<double>(), ctx->J,
                          ctx->P, ctx->Gtmp.as<double>(), ctx->B64.as<double>(), ctx->B32.as<float>(),
                          ctx->stream),
                "fk");
    ART_TRY_HIP(hipMemcpyAsync(B, ctx->B64.p, nb * 8, hipMemcpyDeviceToHost, ctx->stream), "copy");
    ART_TRY_HIP(hipStreamSynchronize(ctx->stream), "fk");
    return ART_OK;
}

art_status art_get_posed_keys(art_ctx* ctx, int pose, unsigned flags, uint32_t* keys) {
    if (!ctx) return ART_EINVAL;
    if (!keys) return fail(ctx, ART_EINVAL, "keys is NULL");
    art_status rc = check_build_state(ctx);
    if (rc != ART_OK) return rc;
    if (pose < 0 || pose >= ctx->P) return fail(ctx, ART_EINVAL, "pose out of range");
    if (flags & ~ART_GEOM_FP32) return fail(ctx, ART_EINVAL, "unknown flag bits");
    DeviceGuard g(ctx->device);
    const size_t nb = (size_t)ctx->P * ctx->J * 12;
    {
        const art_status rb = ensure_bufs(ctx, {{&ctx->B64, nb * 8}, {&ctx->B32, nb * 4}, {&ctx->Gtmp, nb * 8}});
        if (rb != ART_OK) return rb;
    }
    hipStream_t st = ctx->stream;
    ART_TRY_HIP(launch_fk(ctx->parent.as<int32_t>(), ctx->rest.as<double>(), ctx->pose.as<double>(), ctx->J,
                          ctx->P, ctx->Gtmp.as<double>(), ctx->B64.as<double>(), ctx->B32.as<float>(), st),
                "fk");
    ART_TRY_HIP(launch_skin(ctx->ijk.as<uint16_t>(), ctx->bone.as<uint8_t>(), ctx->weight.as<float>(), ctx->n,
                            ctx->depth, ctx->B64.as<double>() + (size_t)pose * ctx->J * 12,
                            ctx->B32.as<float>() + (size_t)pose * ctx->J * 12, ctx->J,
                            (flags & ART_GEOM_FP32) != 0, 1, keys, nullptr, nullptr, 0u, nullptr, st),
                "skin");
    ART_TRY_HIP(hipStreamSynchronize(st), "skin");
    return ART_OK;
}

art_status art_get_octree(art_ctx* ctx, int pose, unsigned flags, int64_t* counts, uint32_t* keys,
                          uint32_t* winner, uint32_t* brick_keys, uint32_t* brick_row, uint32_t* brick_mask) {
    if (!ctx) return ART_EINVAL;
    if (!counts) return fail(ctx, ART_EINVAL, "counts is NULL");
    art_status rc = check_build_state(ctx);
    if (rc != ART_OK) return rc;
    if (pose < 0 || pose >= ctx->P) return fail(ctx, ART_EINVAL, "pose out of range");
    if (flags & ~ART_GEOM_FP32) return fail(ctx, ART_EINVAL, "unknown flag bits");
    DeviceGuard g(ctx->device);
    CallPlan pl;
    pl.C = 4;
    pl.storage = 0;
    pl.fp32 = (flags & ART_GEOM_FP32) != 0;
    pl.Vg = 1;
    pl.ngroups = 1;
    rc = ensure_scratch(ctx, pl, 1);
    if (rc != ART_OK) return rc;
    DevBuf zs, zf;   // the build also permutes a FLUT; feed it zeros
    ART_TRY_HIP(zs.ensure((size_t)ctx->n * 4), "device allocation");
    hipError_t e = zf.ensure((size_t)ctx->n * 16);
    if (e != hipSuccess) {
        zs.release();
        return hip_fail(ctx, e, "device allocation");
    }
    hipStream_t st = ctx->stream;
    e = launch_fill_u32(zs.as<uint32_t>(), 0u, (size_t)ctx->n, st);
    if (e == hipSuccess) e = launch_fill_u32(zf.as<uint32_t>(), 0u, (size_t)ctx->n * 4, st);
    if (e == hipSuccess)
        e = launch_fk(ctx->parent.as<int32_t>(), ctx->rest.as<double>(), ctx->pose.as<double>(), ctx->J, ctx->P,
                      ctx->Gtmp.as<double>(), ctx->B64.as<double>(), ctx->B32.as<float>(), st);
    if (e != hipSuccess) {
        zs.release();
        zf.release();
        return hip_fail(ctx, e, "octree");
    }
    Timing tm;
    int launches = 0;
    rc = build_batch(ctx, pl, pose, 1, zs.p, zf.p, &launches, tm, true);
    PoseCounters hc{};
    if (rc == ART_OK) {
        e = hipMemcpyAsync(&hc, ctx->s.counters.p, sizeof(hc), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(ctx, e, "octree");
    }
    if (rc == ART_OK) {
        counts[0] = hc.M;
        counts[1] = hc.nb;
        counts[2] = hc.dropped;
        counts[3] = ctx->n - hc.dropped - hc.M;
        const Scratch& s = ctx->s;
        if (keys) e = hipMemcpyAsync(keys, s.occ_key.p, (size_t)hc.M * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && winner)
            e = hipMemcpyAsync(winner, s.occ_win.p, (size_t)hc.M * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && brick_keys)
            e = hipMemcpyAsync(brick_keys, s.brick_key.p, (size_t)hc.nb * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && brick_row)
            e = hipMemcpyAsync(brick_row, s.brick_row.p, (size_t)hc.nb * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && brick_mask)
            e = hipMemcpyAsync(brick_mask, s.brick_mask.p, (size_t)hc.nb * 64, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(ctx, e, "octree copy");
    }
    zs.release();
    zf.release();
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Training-side calls: proposal margin calibration, proposal state file, map loss
// ---------------------------------------------------------------------------
namespace {

// Late start of the proposed entry, in leaf edges h, of each ray whose label
// holds a sample (u_near <= u_far): (predicted - labelled u_near) times the
// ray's span inside the posed root [-1, 1]^3 (from max(t_entry, 0) to t_exit),
// over h; NaN for rays without a sample.
__global__ __launch_bounds__(256) void k_calib_late(const float* __restrict__ od, const float* __restrict__ target,
                                                    const float* __restrict__ pred, int64_t n, double h,
                                                    float* __restrict__ late) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float un = target[2 * i], uf = target[2 * i + 1];
    if (!(un <= uf)) {
        late[i] = __builtin_nanf("");
        return;
    }
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double o = od[6 * i + a], d = od[6 * i + 3 + a];
        if (d == 0.0) continue;
        const double t0 = (-1.0 - o) / d, t1 = (1.0 - o) / d;
        lo = fmax(lo, fmin(t0, t1));
        hi = fmin(hi, fmax(t0, t1));
    }
    const double span = hi - fmax(lo, 0.0);
    late[i] = (float)(((double)pred[2 * i] - (double)un) * span / h);
}

// L2 map loss: d = (x - y) * inv_r into dx, per-block partial sums of
// (x - y)^2 (FP64) into part[blockIdx.x].
__global__ __launch_bounds__(256) void k_map_loss(const float* __restrict__ x, const float* __restrict__ y,
                                                  int64_t n, float inv_r, float* __restrict__ dx,
                                                  double* __restrict__ part) {
    __shared__ double red[256 / kWave];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float e = x[i] - y[i];
        dx[i] = e * inv_r;
        acc += (double)e * (double)e;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_down(acc, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

constexpr int kLossBlocks = 1024;

// Sum of (x - y)^2 over n elements (FP64, fixed order) and dx = (x - y) inv_r.
art_status map_loss_part(art_ctx* ctx, const float* x, const float* y, int64_t n, float inv_r, float* dx,
                         double* sum) {
    *sum = 0.0;
    if (n == 0) return ART_OK;
    hipStream_t st = ctx->stream;
    int64_t blocks = (n + 255) / 256;
    if (blocks > kLossBlocks) blocks = kLossBlocks;
    art_status rc = ensure_bufs(ctx, {{&ctx->mlp_calib, (size_t)kLossBlocks * 8}});
    if (rc != ART_OK) return rc;
    hipLaunchKernelGGL(k_map_loss, dim3((unsigned)blocks), dim3(256), 0, st, x, y, n, inv_r, dx,
                       ctx->mlp_calib.as<double>());
    ART_TRY_HIP(hipGetLastError(), "map loss");
    std::vector<double> part((size_t)blocks);
    ART_TRY_HIP(hipMemcpyAsync(part.data(), ctx->mlp_calib.p, (size_t)blocks * 8, hipMemcpyDeviceToHost, st), "copy");
    ART_TRY_HIP(hipStreamSynchronize(st), "map loss");
    for (double v : part) *sum += v;
    return ART_OK;
}

constexpr char kPropMagic[8] = {'A', 'R', 'T', 'P', 'R', 'O', 'P', '1'};

}  // namespace

extern "C" {

art_status art_proposal_calibrate(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, const float* target,
                                  float quantile, float floor_h, float* margin_h) {
    if (!ctx) return ART_EINVAL;
    if (!margin_h) return fail(ctx, ART_EINVAL, "margin_h is NULL");
    if (n < 0 || (n > 0 && (!od || !pose || !target))) return fail(ctx, ART_EINVAL, "n < 0 or NULL buffer");
    if (!(quantile >= 0.0f && quantile <= 1.0f)) return fail(ctx, ART_EINVAL, "quantile must be in [0, 1]");
    if (!(floor_h >= 0.0f) || !std::isfinite(floor_h)) return fail(ctx, ART_EINVAL, "floor_h must be finite, >= 0");
    if (ctx->depth <= 0) return fail(ctx, ART_ESTATE, "no octree loaded (art_load_octree)");
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    *margin_h = floor_h;
    if (n == 0) return ART_OK;
    art_status rc = ensure_bufs(ctx, {{&ctx->mlp_calib, (size_t)n * 12}});
    if (rc != ART_OK) return rc;
    float* pred = ctx->mlp_calib.as<float>();   // [n][2], then the late starts [n]
    float* late = pred + 2 * n;
    rc = art_proposal_forward(ctx, n, od, pose, pred);
    if (rc != ART_OK) return rc;
    const double h = 1.0 / (double)(1 << ctx->depth);
    hipLaunchKernelGGL(k_calib_late, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, od, target, pred, n, h, late);
    ART_TRY_HIP(hipGetLastError(), "calibration");
    std::vector<float> v((size_t)n);
    ART_TRY_HIP(hipMemcpyAsync(v.data(), late, (size_t)n * 4, hipMemcpyDeviceToHost, st), "copy");
    ART_TRY_HIP(hipStreamSynchronize(st), "calibration");
    v.erase(std::remove_if(v.begin(), v.end(), [](float x) { return std::isnan(x); }), v.end());
    if (v.empty()) return ART_OK;
    // quantile with linear interpolation between the order statistics
    std::sort(v.begin(), v.end());
    const double pos = (double)quantile * (double)(v.size() - 1);
    const size_t k = (size_t)pos;
    const double frac = pos - (double)k;
    double q = v[k];
    if (k + 1 < v.size()) q += frac * ((double)v[k + 1] - (double)v[k]);
    *margin_h = (float)std::max((double)floor_h, q);
    return ART_OK;
}

art_status art_proposal_io(art_ctx* ctx, int save, const char* path) {
    if (!ctx) return ART_EINVAL;
    if (!path) return fail(ctx, ART_EINVAL, "path is NULL");
    if (ctx->J <= 0) return fail(ctx, ART_ESTATE, "no skeleton (art_set_skeleton)");
    const MlpDims m = mlp_dims(ctx->J);
    const size_t np = (size_t)m.np;
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    std::vector<float> buf(3 * np);
    if (save) {
        if (ctx->mlp_J != ctx->J)
            return fail(ctx, ART_ESTATE, "no proposal weights for the current skeleton (art_proposal_set_weights)");
        ART_TRY_HIP(hipMemcpyAsync(buf.data(), ctx->mlp_theta.p, np * 4, hipMemcpyDeviceToHost, st), "copy");
        ART_TRY_HIP(hipMemcpyAsync(buf.data() + np, ctx->mlp_m1.p, np * 4, hipMemcpyDeviceToHost, st), "copy");
        ART_TRY_HIP(hipMemcpyAsync(buf.data() + 2 * np, ctx->mlp_m2.p, np * 4, hipMemcpyDeviceToHost, st), "copy");
        ART_TRY_HIP(hipStreamSynchronize(st), "copy");
        FILE* f = fopen(path, "wb");
        if (!f) return fail(ctx, ART_EINVAL, std::string("cannot open ") + path + " for writing");
        const int32_t hdr[2] = {ctx->J, 0};
        const int64_t cnt[2] = {m.np, ctx->mlp_step};
        bool ok = fwrite(kPropMagic, 1, 8, f) == 8 && fwrite(hdr, 4, 2, f) == 2 && fwrite(cnt, 8, 2, f) == 2 &&
                  fwrite(buf.data(), 4, 3 * np, f) == 3 * np;
        ok = (fclose(f) == 0) && ok;
        if (!ok) return fail(ctx, ART_EINVAL, std::string("write to ") + path + " failed");
        return ART_OK;
    }
    FILE* f = fopen(path, "rb");
    if (!f) return fail(ctx, ART_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t hdr[2];
    int64_t cnt[2];
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kPropMagic, 8) == 0 && fread(hdr, 4, 2, f) == 2 &&
              fread(cnt, 8, 2, f) == 2;
    ok = ok && hdr[0] == ctx->J && cnt[0] == m.np && cnt[1] >= 0 && fread(buf.data(), 4, 3 * np, f) == 3 * np;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;   // nothing after the state
    fclose(f);
    if (!ok) return fail(ctx, ART_EINVAL, std::string(path) + " is not a proposal state for J = " + std::to_string(ctx->J));
    for (size_t i = 0; i < 3 * np; ++i)
        if (!std::isfinite(buf[i]) || (i >= 2 * np && buf[i] < 0.0f))
            return fail(ctx, ART_EINVAL, std::string(path) + ": non-finite value or negative second moment");
    const size_t bytes = np * 4;
    art_status rc = ensure_bufs(ctx, {{&ctx->mlp_theta, bytes}, {&ctx->mlp_m1, bytes}, {&ctx->mlp_m2, bytes}});
    if (rc != ART_OK) return rc;
    ART_TRY_HIP(hipMemcpyAsync(ctx->mlp_theta.p, buf.data(), bytes, hipMemcpyHostToDevice, st), "copy");
    ART_TRY_HIP(hipMemcpyAsync(ctx->mlp_m1.p, buf.data() + np, bytes, hipMemcpyHostToDevice, st), "copy");
    ART_TRY_HIP(hipMemcpyAsync(ctx->mlp_m2.p, buf.data() + 2 * np, bytes, hipMemcpyHostToDevice, st), "copy");
    ART_TRY_HIP(hipStreamSynchronize(st), "copy");
    ctx->mlp_J = ctx->J;
    ctx->mlp_step = cnt[1];
    return ART_OK;
}

art_status art_map_loss(art_ctx* ctx, int64_t n_feat, int64_t rays, const float* F, const float* F_target,
                        const float* A, const float* A_target, float* d_feat, float* d_alpha, double* loss) {
    if (!ctx) return ART_EINVAL;
    if (!loss) return fail(ctx, ART_EINVAL, "loss is NULL");
    if (n_feat < 0 || rays < 1) return fail(ctx, ART_EINVAL, "n_feat >= 0 and rays >= 1");
    if (n_feat > 0 && (!F || !F_target || !d_feat)) return fail(ctx, ART_EINVAL, "NULL feature buffer");
    if (A_target && (!A || !d_alpha)) return fail(ctx, ART_EINVAL, "NULL opacity buffer");
    DeviceGuard g(ctx->device);
    const float inv_r = (float)(1.0 / (double)rays);
    double sf = 0.0, sa = 0.0;
    art_status rc = map_loss_part(ctx, F, F_target, n_feat, inv_r, d_feat, &sf);
    if (rc != ART_OK) return rc;
    if (A_target) {
        rc = map_loss_part(ctx, A, A_target, rays, inv_r, d_alpha, &sa);
        if (rc != ART_OK) return rc;
    }
    *loss = 0.5 * (sf + sa) / (double)rays;
    return ART_OK;
}

art_status art_render_status(art_ctx* ctx, int64_t* overflowed_items, int64_t* bad_densities) {
    if (!ctx) return ART_EINVAL;
    int64_t ov = 0, bad = 0;
    if (ctx->async_pending) {
        DeviceGuard g(ctx->device);
        hipStream_t st = ctx->stream;
        const size_t items = ctx->async_items;
        std::vector<uint32_t> hov(items * 2);
        unsigned long long hst[16] = {0};
        ART_TRY_HIP(hipMemcpyAsync(hov.data(), ctx->s.ovf.p, items * 2 * 4, hipMemcpyDeviceToHost, st), "copy");
        ART_TRY_HIP(hipMemcpyAsync(hst, ctx->s.stats.p, sizeof(hst), hipMemcpyDeviceToHost, st), "copy");
        ART_TRY_HIP(hipStreamSynchronize(st), "render status");
        size_t need = 0;
        for (size_t i = 0; i < items; ++i) {
            ctx->s.pair_hint = std::max<size_t>(ctx->s.pair_hint, hov[2 * i + 1]);
            if (hov[2 * i] != 0u && hov[2 * i + 1] > ctx->s.pair_cap) {
                ++ov;
                need = std::max<size_t>(need, hov[2 * i + 1]);
            }
        }
        // the next call's tile lists hold what this one needed
        if (need) ctx->s.pair_cap = need + need / 4 + 1024;
        bad = (int64_t)hst[kStatBadSigma];
        for (int i = 0; i < 7; ++i) ctx->stats[i] = (int64_t)hst[i];
        ctx->stats[7] = ctx->async_launches;
        for (int i = 8; i < 15; ++i) ctx->stats[i] = (int64_t)hst[i - 1];
        ctx->async_pending = false;
        // a complete build may be reused (ART_REUSE_BUILD) as after a synchronous call
        if (ctx->async_memo.valid && ov == 0 && bad == 0) ctx->memo = ctx->async_memo;
        ctx->async_memo.valid = false;
    }
    if (overflowed_items) *overflowed_items = ov;
    if (bad_densities) *bad_densities = bad;
    return ART_OK;
}

art_status art_get_stats(art_ctx* ctx, int64_t* stats) {
    if (!ctx) return ART_EINVAL;
    if (!stats) return fail(ctx, ART_EINVAL, "stats is NULL");
    for (int i = 0; i < kNumStats; ++i) stats[i] = ctx->stats[i];
    return ART_OK;
}

art_status art_get_timing(art_ctx* ctx, float* ms, int* n_render) {
    if (!ctx) return ART_EINVAL;
    if (!ms) return fail(ctx, ART_EINVAL, "ms is NULL");
    if (!ctx->timing_valid) return fail(ctx, ART_ESTATE, "no call with ART_TIMING yet");
    for (int i = 0; i < 7; ++i) ms[i] = ctx->timing_ms[i];
    if (n_render) *n_render = ctx->timing_nrender;
    return ART_OK;
}

}  // extern "C"
