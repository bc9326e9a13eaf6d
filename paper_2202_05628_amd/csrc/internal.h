// Host-side internals of libartemis: context, device buffers, launcher
// declarations.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/artemis.h"
#include "validate.h"

namespace art {

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) {
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = bytes < 256 ? 256 : bytes;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        else p = nullptr;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};


// Parameter layout of the proposal network for J bones (flat FP32 vector:
// W1 [64][n_in], b1, W2 [64][64], b2, W3 [64][64], b3, W4 [2][64], b4).
// Loss of the proposal network: 0 SmoothL1 (beta = 1); 1 one-sided: pinball
// at levels tau[0] (u_near) and tau[1] (u_far) on rays whose label holds a
// sample, SmoothL1 on rays with the empty label.
struct MlpLoss {
    int kind = 0;
    float tau[2] = {0.5f, 0.5f};
};

struct MlpDims {
    int J, n_in, np;
    int oW1, ob1, oW2, ob2, oW3, ob3, oW4, ob4;
};
inline MlpDims mlp_dims(int J) {
    MlpDims m;
    m.J = J;
    m.n_in = 6 + 6 * J;
    m.oW1 = 0;
    m.ob1 = m.oW1 + 64 * m.n_in;
    m.oW2 = m.ob1 + 64;
    m.ob2 = m.oW2 + 64 * 64;
    m.oW3 = m.ob2 + 64;
    m.ob3 = m.oW3 + 64 * 64;
    m.oW4 = m.ob3 + 64;
    m.ob4 = m.oW4 + 2 * 64;
    m.np = m.ob4 + 2;
    return m;
}

// Device-side counters of one pose (written by the build kernels).
struct PoseCounters {
    uint32_t M;          // occupied posed cells
    uint32_t nb;         // bricks
    uint32_t dropped;    // leaves outside the posed root
    uint32_t npairs;     // tile/brick pairs
    uint32_t overflow;   // pair buffer overflow flag
    uint32_t pad[3];
};

// Run-wide statistics accumulated on the device.
struct RunStats {
    unsigned long long rays, samples, hit_rays, dropped, collisions, bricks, pairs, list_entries, rounds,
        steps, tile_rays;
};

constexpr int kNumStats = 15;
constexpr int kStatBadSigma = 15;     // device run-statistics slot: FLUT densities < 0 or not finite
constexpr int kMaxBonesSH = 64;       // bone rotations staged in LDS by the view-dependent (SH) render
constexpr int kSortBlocks = 512;      // fixed grid (per pose) of the radix-sort passes
constexpr int kScanBlocks = 256;      // fixed grid (per pose) of device-sized scans
constexpr int kUniqueBlocks = 512;    // fixed grid (per pose) of the unique / compaction step

struct Scratch {
    DevBuf keys0, keys1;                 // [slots][n] posed key / posed row of each leaf
    DevBuf hist, digit_tot;              // [slots][256 * kSortBlocks], [slots][256]
    DevBuf blk0, blk1;                   // block partials [slots][max(kScanBlocks, kUniqueBlocks)]
    DevBuf bmap, wpref;                  // [slots][bwords] brick occupancy bits, bricks before each word
    DevBuf occ_key, occ_win;             // [slots][n] posed cells + winners
    DevBuf brick_key, brick_row, brick_mask;  // [slots][n], [slots][n+1], [slots][n*16]
    DevBuf bin_cnt, bin_off;             // [slots][n * Vg]
    size_t bin_stride = 0;               // n * Vg
    DevBuf pk0, pk1;                     // pair sort keys [slots][pair_cap]
    DevBuf pv0;                          // pair sort payload scratch [slots][groups][pair_cap]
    DevBuf pair_v;                       // [slots][groups][pair_cap] sorted brick ids
    DevBuf tile_start, tile_end;         // [slots][V][tiles]
    DevBuf counters;                     // PoseCounters [slots]
    DevBuf stats;                        // RunStats
    DevBuf ovf;                          // [slots][groups][2] overflow flag, pair count
    DevBuf items;                        // [slots][V][tiles] compacted non-empty tiles
    DevBuf redo;                         // [slots][groups] items re-run after an overflow
    DevBuf queue;                        // [2] item count, queue head
    DevBuf loss;                         // [1] double: loss accumulator of the training-step kernels
    DevBuf interval;                     // [slots][V][tiles][64] float2 proposed intervals
    size_t pair_cap = 0;
    size_t pair_hint = 0;                // largest tile-list length seen (sizes the list sort's grid)
    int slots = 0;                       // poses whose octrees are held at once
};

}  // namespace art

struct art_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // canonical octree + skin
    int depth = 0;
    int64_t n = 0;
    art::DevBuf ijk;      // uint16 [3][n]
    art::DevBuf bone;     // uint8 [4][n]
    art::DevBuf weight;   // float [4][n]
    art::DevBuf dom_bone; // uint8 [n]: bone of each leaf's largest skin weight

    // shading network: FP16 conv weights [3][3][Cout][Cin] per layer, FP32
    // biases, FP32 head; activation scratch
    int shade_C = 0;
    art::DevBuf shade_w, shade_b, shade_head;
    art::DevBuf shade_act;
    void* shade_fixed = nullptr;   // device address of the fixed activation array on this device
    bool has_skin = false;
    int max_bone = -1;

    // skeleton
    int J = 0;
    art::DevBuf parent;   // int32 [J]
    art::DevBuf rest;     // double [J][3]

    // poses
    int P = 0;
    art::DevBuf pose;     // double [P][J+2][3]  (r_0..r_{J-1}, R, T)

    // cameras
    int V = 0, H = 0, W = 0;
    std::vector<art::CamParams> cams;
    art::DevBuf cam;      // CamParams [V]

    // derived
    art::DevBuf B64, B32, Gtmp;

    art::Scratch s;

    // learned ray-interval proposal
    int mlp_J = 0;                 // skeleton size the weights were set for (0: none)
    int64_t mlp_step = 0;          // Adam steps taken since the weights were set
    art::MlpLoss mlp_loss_fn;      // training loss (art_proposal_set_loss)
    art::DevBuf mlp_theta, mlp_m1, mlp_m2;   // FP32 master weights and Adam moments
    art::DevBuf mlp_packed;        // BF16 matrix-core operands
    art::DevBuf mlp_cbias;         // [P][64] per-pose first-layer bias
    art::DevBuf mlp_code;          // [P][6J] pose codes
    art::DevBuf mlp_S, mlp_part, mlp_lossp, mlp_loss, mlp_flag;
    art::DevBuf mlp_calib;         // margin calibration and map-loss scratch
    int64_t poses_version = 0;     // bumped by art_set_poses
    int64_t code_version = -1;     // poses_version the pose codes were computed for

    // timing events of the stages, reused by every call that asks for timings
    std::vector<hipEvent_t> ev_pool;

    // The posed octrees and tile lists a render call leaves in the scratch
    // slots, for an adjoint or VRT call that asks to reuse them (they depend
    // only on the octree, skin, skeleton, poses, cameras and the geometry
    // precision, not on the FLUT).  Every setter bumps state_version; every
    // build clears `valid`; a reallocated scratch buffer changes its pointers.
    uint64_t state_version = 0;
    size_t mem_limit = 0;          // bound on the working buffers' total capacity (0: none)
    // last call made with ART_ASYNC whose overflow flags and statistics were
    // not read back yet (art_render_status)
    bool async_pending = false;
    size_t async_items = 0;
    int async_launches = 0;
    struct BuildMemo {
        bool valid = false;
        uint64_t version = 0;
        bool fp32 = false;
        int P = 0, Vg = 0, ngroups = 0, H = 0, W = 0;
        size_t pair_cap = 0;
        const void* occ = nullptr;     // s.occ_win.p when the memo was taken
        const void* lists = nullptr;   // s.pair_v.p
        const void* rows = nullptr;    // s.keys1.p
        const void* tiles = nullptr;   // s.tile_start.p
        const void* counters = nullptr;   // s.counters.p
    } memo;
    // the build of the last ART_ASYNC call, made the memo by art_render_status
    // when none of its items overflowed
    BuildMemo async_memo;

    // last-call bookkeeping
    int64_t stats[art::kNumStats] = {0};
    float timing_ms[7] = {0};
    int timing_nrender = 0;
    bool timing_valid = false;
};

namespace art {

// ---- launchers (each enqueues on `st`) ------------------------------------
// Kernels of the octree build run for a batch of poses at once (pose =
// blockIdx.y); per-pose arrays are addressed as base + pose * stride.
hipError_t launch_fk(const int32_t* parent, const double* rest, const double* pose, int J, int P,
                     double* G, double* B64, float* B32, hipStream_t st);
hipError_t launch_skin(const uint16_t* ijk, const uint8_t* bone, const float* w, int64_t n,
                       int depth, const double* B64, const float* B32, int J, bool fp32, int batch,
                       uint32_t* keys, uint32_t* vals, uint32_t* bmap, uint32_t bwords, PoseCounters* cnt,
                       hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);

struct SortBatch {
    uint32_t *k0, *k1;    // keys (ping-pong), pose stride kstride
    uint32_t *v0, *v1;    // payloads (ping-pong), pose stride vstride
    size_t kstride, vstride;
    const uint32_t* d_n;  // item count of pose p at d_n[p * nstride]
    uint32_t nstride;
    uint32_t n_cap;       // largest item count (sizes the grid)
    uint32_t* hist;       // [batch][256 * kSortBlocks]
    uint32_t* digit_tot;  // [batch][256]
    int batch;
};
hipError_t launch_radix_sort(const SortBatch& b, int bits, hipStream_t st, bool* result_in_1, int* launches);
hipError_t launch_scan_exclusive(const uint32_t* in, uint32_t* out, size_t stride, const uint32_t* d_n,
                                 uint32_t nstride, uint32_t* d_total, uint32_t tstride, uint32_t* blk, int batch,
                                 hipStream_t st, int* launches);

// Posed octrees of a batch of poses (slot p at base + p * stride).
struct OctreeSlot {
    uint32_t* occ_key;      // [n]
    uint32_t* occ_win;      // [n]
    uint32_t* brick_key;    // [n]
    uint32_t* brick_row;    // [n + 1]
    uint32_t* brick_mask;   // [n][16]
};
// Words of the brick occupancy bitmap of a posed lattice of depth + 1.
inline uint32_t brick_words(int depth) {
    const int bits = 3 * (depth + 1) - 9;   // bits of a brick key (key >> 9)
    return bits <= 5 ? 1u : (1u << (bits - 5));
}
// Octree build from the unsorted posed keys of a batch (keys + pose * n, the
// invalid key for dropped leaves) and the brick bitmap the skinning marked.
hipError_t launch_build_octree_dense(const uint32_t* keys, uint32_t n, int depth, Scratch& s, const OctreeSlot& o,
                                     int batch, hipStream_t st, int* launches);
int bin_key_bits(int Vg, int H, int W, int depth, int* mbits);
// Tile lists of views [v0, v0 + Vg) of every pose of the batch: sorted brick
// ids into pair_v + (p * ngroups + group) * pair_cap, per-tile ranges into
// tile_start / tile_end + (p * V + v0) * TPV.
hipError_t launch_bin(Scratch& s, const CamParams* cam_dev, const OctreeSlot& o, size_t n, int batch, int V, int v0,
                      int Vg, int group, int ngroups, int H, int W, int depth, bool fp32, hipStream_t st,
                      int* launches);
__global__ void k_pairs(const PoseCounters* __restrict__ c, unsigned long long* __restrict__ st,
                        uint32_t* __restrict__ ovf, int ngroups, int group, const uint8_t* __restrict__ redo,
                        int batch);

struct RenderLaunch {
    int C, storage;
    bool fp32;
    int mode;            // 0 forward, 1 backward, 2 debug hit lists, 3 labels, 4 proposal, 5 forward + depth,
                         // 6 forward with SH features
    int depth;
    bool bg_in_render;   // the compositing kernel also writes the background pixels
    int Pb, V, H, W;     // poses in the launch (slots 0..Pb-1), views, image
    int Vg, ngroups;     // view groups of the tile lists
    uint32_t ncap;       // leaves per slot
    float lambda;
    const CamParams* cam;
    const Scratch* s;
    const void* sigma;   // canonical FLUT (device)
    const void* feat;
    // maps of the launch's first pose (pose offset applied by the caller)
    float* out_feat;
    float* out_alpha;
    float* out_tfinal;
    const float* fwd_feat;
    const float* fwd_tfinal;
    const float* d_feat;
    const float* d_alpha;
    float* d_sigma;
    float* d_leaf_feat;
    float* labels;           // [Pb][V][H][W][2] (mode 3)
    const float* interval;   // [Pb][V][H][W][2], or [items][64][2] with interval_by_item (mode 4)
    bool interval_by_item;
    float margin;            // ray-parameter units
    float f2_tau;
    bool near_only;          // mode 4: the interval ends at t_b
    float* out_depth;        // [Pb][V][H][W] (mode 5)
    float depth_sigma;       // density threshold of the depth buffer
    int sh_H;                // SH coefficients per leaf (mode 6)
    int J;
    const uint8_t* dom_bone; // [n] (mode 6)
    const float* bone_rot;   // [Pb][J][12] bone transforms of the launch's poses (mode 6)
    int max_hits;
    int debug_view;
    int32_t* hit_leaf;
    double* hit_delta;
    int32_t* hit_count;
    float* ckpt;             // ray checkpoints of the launch's first map (mode 7 writes, mode 1 reads)
    int32_t* ckpt_n;
    int ckpt_K, ckpt_every;  // records per ray, samples per segment (0: none)
};
hipError_t launch_render(const RenderLaunch& r, hipStream_t st);
int num_cus();   // compute units of the current device

// Tile compaction (non-empty tiles -> work list) and background of empty tiles.
struct TileLaunch {
    int Pb, V, Vg, ngroups, H, W, C;
    uint32_t tiles_pow4;
    int debug_view;            // -1: all views
    const uint32_t* ovf;
    const uint32_t* tile_start;
    const uint32_t* tile_end;
    uint32_t* items;           // [Pb * V * TPV]
    uint32_t* counters;        // [2]: item count, queue head
    float* out_feat;           // forward maps (null in the adjoint)
    float* out_alpha;
    float* out_tfinal;
    float* labels;             // interval labels (label pass)
    float* out_depth;          // depth buffer (+inf on empty tiles)
    int32_t* hit_count;
    unsigned long long* stats;
    bool bg_in_render;         // the compositing kernel writes the background (vectorised maps only)
};
hipError_t launch_tiles(const TileLaunch& t, hipStream_t st);
// Whether the launch's maps take the vectorised background (width a multiple
// of 4, 16-byte aligned maps).
bool background_vectorised(const TileLaunch& t);

// Proposal network (k_mlp.hip).
struct AdamStep {
    float lr, beta1, beta2, eps, bc1, bc2;   // bc = 1 - beta^step
};
// FLUT training step (k_train.hip).  rows: [batch][n] posed row of each leaf
// from the octree build (kInvalidKey for dropped leaves).
hipError_t launch_vrt(const uint32_t* rows, const uint32_t* occ_win, uint32_t n, int C, int storage,
                      const void* feat, const PoseCounters* cnt, float lambda, int batch, float* d_feat,
                      double* loss, hipStream_t st);
hipError_t launch_query(const double* pts, int64_t n, int depth, const OctreeSlot& o, const PoseCounters* cnt,
                        int32_t* out, hipStream_t st);
hipError_t launch_flut_adam(float* param, const float* grad, float* m, float* v, int64_t count, const AdamStep& a,
                            float lower, hipStream_t st);
// Shading network (k_shade.hip).  FP16 tensors are passed as uint16_t.
struct ConvLaunch {
    const uint16_t* src1;   // NHWC [N][H][W][C1]
    int C1;                 // multiple of 32
    const uint16_t* src2;   // NHWC [N][H/2][W/2][C2] read nearest-upsampled, or null (C2 = 0)
    int C2;                 // multiple of 32
    const uint16_t* wgt;    // [3][3][Cout][C1 + C2]
    const float* bias;      // [Cout]
    uint16_t* out;          // NHWC [N][H][W][Cout], Cout a multiple of 32
    int N, H, W, Cout, relu;
};
hipError_t launch_conv3x3(const ConvLaunch& a, hipStream_t st);
hipError_t launch_to_nhwc(const float* F, int N, int C, int H, int W, int Cp, uint16_t* out, hipStream_t st);
hipError_t launch_maxpool2(const uint16_t* in, int N, int H, int W, int C, uint16_t* out, hipStream_t st);
hipError_t launch_head(const uint16_t* in, int N, int H, int W, const float* w, const float* b, float* out,
                       hipStream_t st);
struct InferLaunch {
    const uint16_t* packed;
    const float* theta;
    const float* cbias;
    MlpDims m;
    const CamParams* cam;
    const uint32_t* items;
    const uint32_t* n_items;
    int V, TX, TPV, pose0;
    float* out;            // [items][64] float2
};
hipError_t launch_pose_code(const double* pose, int J, int P, float* code, hipStream_t st);
hipError_t launch_mlp_prep(const float* theta, const MlpDims& m, const float* code, int P, uint16_t* packed,
                           float* cbias, hipStream_t st);
int64_t mlp_pad(int64_t n);
size_t mlp_scratch_bytes(int64_t n);
int mlp_packed_elems();
unsigned mlp_loss_parts(int64_t n);
hipError_t launch_mlp_forward(const uint16_t* packed, const float* theta, const float* cbias, const MlpDims& m,
                              const float* od, const int32_t* pose, int P, int64_t n, float* out, uint32_t* bad,
                              hipStream_t st);
hipError_t launch_mlp_grad(const uint16_t* packed, const float* theta, const float* cbias, const float* code,
                           const MlpDims& m, const float* od, const int32_t* pose, const float* target, int P,
                           int64_t n, float* S, float* part, float* loss_part, uint32_t* bad, const MlpLoss& loss,
                           hipStream_t st);
hipError_t launch_mlp_reduce(const float* part, int64_t n, const MlpDims& m, float* grad, float* theta, float* m1,
                             float* m2, const AdamStep* adam, const float* loss_part, float* loss_out,
                             hipStream_t st);
hipError_t launch_mlp_gather(const int64_t* ray_id, int64_t n, const float* labels, const CamParams* cam, int P,
                             int V, int H, int W, float* od, int32_t* pose, float* target, uint32_t* bad,
                             hipStream_t st);
hipError_t launch_mlp_infer_tiles(const InferLaunch& a, unsigned grid, hipStream_t st);

}  // namespace art
