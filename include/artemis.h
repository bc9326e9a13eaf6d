/*
 * artemis.h - C ABI of the MI355X animated-octree feature renderer.
 *
 * The renderer follows Section 3.1 of Luo et al., "Artemis: Articulated Neural
 * Pets with Appearance and Motion Synthesis" (ACM TOG 41(4), 2022):
 *
 *   canonical octree leaves + FLUT (features and densities)   "Octree Feature Indexing"
 *   -> bone transforms of the skeleton S = {r, R, T}           "Rigging and Deformation"
 *   -> linear blend skinning of every leaf (Eq. 4)
 *   -> rebuild of the posed octree, collisions resolved
 *   -> ray / voxel indexing, front-to-back compositing of
 *      densities and C-channel features (Eq. 5, Eq. 6),
 *      coarse opacity map, early stop at lambda_th           "Dynamic Volume Rendering"
 *
 * plus the adjoint of the compositing step (the pipeline is trained end to
 * end), a BF16 storage form of the FLUT and a learned ray-interval proposal.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status codes only: no call aborts or throws across the ABI.  On failure
 *   art_last_error(ctx) describes the problem and the context keeps its
 *   previous valid state.
 * - "host" pointers are read during the call and may be freed after it
 *   returns; "device" pointers are HIP device memory owned by the caller
 *   (e.g. torch tensors) that must stay valid until the call returns.
 * - Every device write happens on the HIP stream given to art_create.
 *   art_render and art_backward synchronise that stream before returning, so
 *   their outputs are complete when they return - unless called with
 *   ART_ASYNC (see there and art_render_status).
 * - Canonical grid: depth D, 2^D cells per axis over [-1/2, 1/2]^3, leaf edge
 *   h = 2^-D; leaf centre p = -1/2 + (ijk + 1/2) h.
 * - Posed grid: [-1, 1]^3 with the same leaf edge, G = 2^(D+1) cells per axis;
 *   a posed centre p lies in cell floor((p + 1) / h).  Leaves that leave the
 *   posed root are dropped (counted, not an error).
 * - Morton keys interleave the 10-bit x, y, z cell coordinates with x in the
 *   lowest bit: key = sum_b x_b << 3b | y_b << (3b+1) | z_b << (3b+2).
 * - Images are row-major, pixel (x, y) at index y * W + x; maps are planar:
 *   feature maps [P][V][C][H][W], opacity / transmittance maps [P][V][H][W].
 */
#ifndef ARTEMIS_H
#define ARTEMIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct art_ctx art_ctx;

typedef enum {
    ART_OK = 0,
    ART_EINVAL = -1,        /* invalid argument (null, size, range, non-finite)  */
    ART_ENOMEM = -2,        /* device allocation failed                           */
    ART_EDEVICE = -3,       /* HIP runtime / kernel launch error                  */
    ART_ESTATE = -4,        /* call made before the inputs it needs were set      */
    ART_EUNSUPPORTED = -5   /* valid but unsupported configuration (e.g. C)       */
} art_status;

typedef enum { ART_F32 = 0, ART_BF16 = 1 } art_dtype;

/* art_render / art_backward flags */
#define ART_GEOM_FP32 1u   /* FP32 skinning and ray parameter (precision form);
                              default: FP64 skinning arithmetic and ray t      */
#define ART_TIMING 2u      /* record per-stage HIP events, read by art_get_timing */
#define ART_PROPOSAL_NEAR_ONLY 4u  /* art_render_proposal: use only u_near, traverse to t_b */
#define ART_REUSE_BUILD 8u /* art_backward, art_vrt: reuse the posed octrees (and tile
                              lists) the last art_render call on this context left,
                              when that call covered every pose in one batch and
                              nothing they depend on (octree, skin, skeleton, poses,
                              cameras, ART_GEOM_FP32) changed since, and no other
                              call rebuilt them; otherwise they are rebuilt, as
                              without the flag.  The FLUT does not enter them.     */
#define ART_ASYNC 16u      /* render calls and art_backward: enqueue the work and
                              return without synchronising the stream, when the
                              poses fit one batch of the context's working memory
                              (else the call is synchronous).  The call uses the
                              tile-list capacity earlier calls established: a
                              (pose, view group) whose lists overflow is not
                              rendered (its maps are unspecified), and a negative
                              or non-finite density makes the call render
                              nothing, without an error.  art_render_status
                              reports both, and the statistics, for the last
                              call; a later call grows the lists as needed.
                              Excludes ART_TIMING.                                 */

/* Library version (major * 10000 + minor * 100 + patch). */
int art_version(void);

/*
 * Create a context on HIP device `device` that enqueues all work on `stream`
 * (a hipStream_t; NULL for the default stream).  *out receives the context.
 * Errors: ART_EINVAL (out NULL, bad device), ART_EDEVICE (HIP failure).
 */
art_status art_create(int device, void* stream, art_ctx** out);

/* Destroy a context and free its device memory.  NULL-safe. */
void art_destroy(art_ctx* ctx);

/* Message of the last failed call on ctx ("" if none).  Never NULL; ctx may be NULL. */
const char* art_last_error(const art_ctx* ctx);

/*
 * Counter of the inputs the posed octrees depend on: every call of
 * art_load_octree, art_set_skin, art_set_skeleton, art_set_poses and
 * art_set_cameras increments it (even when it fails).  A caller that keeps the
 * outputs of a render for a later art_backward (an autograd graph) records it
 * with the render and checks it before the backward: the adjoint re-traverses
 * the rays of the context's current poses and cameras.  0 for a NULL ctx.
 */
uint64_t art_state_version(const art_ctx* ctx);

/*
 * Bound on the context's working memory: the device buffers the library
 * allocates beyond the copies of its inputs (posed octrees, tile lists, sort
 * and scan scratch, proposal-network state and scratch, shading activations).
 * bytes <= 0 removes the bound (the default).  A call that would grow the
 * working buffers beyond the bound fails with ART_ENOMEM before allocating and
 * leaves the context usable; render calls first shrink their pose batches to
 * fit it.  Buffers already held are not released.
 * art_get_memory: current working bytes and the bound (host int64, either
 * pointer may be NULL).
 * Errors: ART_EINVAL (NULL ctx).
 */
art_status art_set_memory_limit(art_ctx* ctx, int64_t bytes);
art_status art_get_memory(art_ctx* ctx, int64_t* working_bytes, int64_t* limit);

/*
 * Load the canonical octree: the occupied leaf array P of Section 3.1
 * ("Octree Feature Indexing"), as n leaves at depth `depth` (1..9).
 * ijk: host uint16 [3][n] SoA planes (x plane, y plane, z plane), each < 2^depth,
 * no duplicate cells.  Copied to device.  Invalidates skin weights.
 * Errors: ART_EINVAL (depth, n < 1, out-of-range or duplicate cells), ART_ENOMEM.
 */
art_status art_load_octree(art_ctx* ctx, int depth, int64_t n, const uint16_t* ijk);

/*
 * Per-leaf skin weights for Eq. 4: four (bone, weight) pairs per leaf.
 * bone: host uint8 [4][n] SoA planes; weight: host float32 [4][n] SoA planes,
 * finite and >= 0 (used as given, not renormalised).  Copied to device.
 * Bone ids are checked against the skeleton at render time.
 * Errors: ART_ESTATE (no octree), ART_EINVAL, ART_ENOMEM.
 */
art_status art_set_skin(art_ctx* ctx, const uint8_t* bone, const float* weight);

/*
 * Skeleton in its canonical pose (Section 3.1, "Rigging and Deformation"):
 * J joints (1..255), parent: host int32 [J] with parent[0] = -1 and
 * 0 <= parent[j] < j, rest_joint: host float64 [J][3] joint positions.  The
 * canonical bone transforms are M^c_j = [I | rest_joint_j].
 * Errors: ART_EINVAL.
 */
art_status art_set_skeleton(art_ctx* ctx, int J, const int32_t* parent, const double* rest_joint);

/*
 * P target poses (1..4096) of the skeleton parameter S = {r, R, T}:
 * r: host float64 [P][J][3] per-joint axis-angle rotations (radians),
 * R: host float64 [P][3] global axis-angle rotation about joint 0,
 * T: host float64 [P][3] global translation.  Copied.  The posed transforms
 * are G_0 = [Rot(R) Rot(r_0) | J_0 + T], G_j = G_parent [Rot(r_j) | J_j - J_parent],
 * and the skinning matrices of Eq. 4 are B_j = M^t_j (M^c_j)^-1 = G_j [I | -J_j],
 * composed in FP64 on the GPU.
 * Errors: ART_ESTATE (no skeleton), ART_EINVAL (non-finite values).
 */
art_status art_set_poses(art_ctx* ctx, int P, const double* r, const double* R, const double* T);

/*
 * V pinhole cameras (OpenCV convention: x right, y down, z forward; pixel
 * centres at +1/2; one ray per pixel, r_p = (o_p, d_p) of Section 3.1):
 * K: host float64 [V][3][3] intrinsics (fx = K[0][0], fy = K[1][1],
 * cx = K[0][2], cy = K[1][2]; skew ignored), c2w: host float64 [V][3][4]
 * camera-to-world [R | t]; the ray origin is t and the direction is
 * normalize(R ((x + 1/2 - cx)/fx, (y + 1/2 - cy)/fy, 1)).  H, W in 1..8192.
 * Errors: ART_EINVAL.
 */
art_status art_set_cameras(art_ctx* ctx, int V, int H, int W, const double* K, const double* c2w);

/*
 * Render every (pose, view): FK -> skinning -> posed octree rebuild -> ray
 * indexing -> compositing (Eq. 5-6) with the early stop of Section 3.1 (stop
 * right after the sample at which the transmittance falls below lambda_th;
 * lambda_th = 0 disables it; the paper uses 0.01).
 *
 * C: feature channels, one of 4, 8, 16, 32.
 * dtype: storage of the FLUT (ART_F32 or ART_BF16; BF16 is converted to FP32
 *        on load, transmittance and accumulation are always FP32).
 * sigma: device [n] densities of the canonical leaves, in dtype; every one
 *        finite and >= 0 (checked on the device: otherwise the call renders
 *        nothing, returns ART_EINVAL, and the outputs are unspecified).  The
 *        features are not checked: a non-finite feature reaches the maps of
 *        the pixels that composite it.
 * feat:  device [n][C] features of the canonical leaves, in dtype (row-major).
 * out_feat:   device float32 [P][V][C][H][W] feature maps F.
 * out_alpha:  device float32 [P][V][H][W] coarse opacity maps A (sum of weights).
 * out_tfinal: device float32 [P][V][H][W] final transmittance, or NULL.
 * Pixels whose ray meets no occupied voxel get F = 0, A = 0, T = 1.
 * Collisions: when several leaves warp into one posed cell the one with the
 * smallest canonical index is rendered.
 * Errors: ART_ESTATE (octree, skin, skeleton, poses or cameras missing),
 * ART_EINVAL (null pointers, lambda_th outside [0,1), bone id >= J, a
 * negative or non-finite density),
 * ART_EUNSUPPORTED (C), ART_ENOMEM, ART_EDEVICE.
 */
art_status art_render(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                      float lambda_th, unsigned flags,
                      float* out_feat, float* out_alpha, float* out_tfinal);

/*
 * Adjoint of art_render for the same poses, cameras, FLUT, lambda_th and
 * flags.  Each ray is re-traversed (no stored sample lists); the composited
 * samples are held fixed at those of the forward pass.
 *
 * out_feat, out_tfinal: device float32 outputs of the forward call.
 * d_feat:  device float32 [P][V][C][H][W] dL/dF.
 * d_alpha: device float32 [P][V][H][W] dL/dA, or NULL for zero.
 * d_sigma: device float32 [n], accumulated (+=) with dL/dsigma.
 * d_leaf_feat: device float32 [n][C], accumulated (+=) with dL/df.
 * Gradients reach only collision winners; dropped and hidden leaves get 0.
 * Float atomics make the summation order, and so the last bits, vary.
 * flags: as art_render, plus ART_REUSE_BUILD (skip the octree rebuild when the
 * last art_render's octrees still apply).
 * Errors: as art_render.
 */
art_status art_backward(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                        float lambda_th, unsigned flags,
                        const float* out_feat, const float* out_tfinal,
                        const float* d_feat, const float* d_alpha,
                        float* d_sigma, float* d_leaf_feat);

/*
 * Segmented adjoint.  The adjoint's time on a launch with fewer 8x8 tiles
 * than the GPU has wave slots is the serial chain of its longest rays (one
 * sample after the other, Eq. 5-6).  art_render_ckpt renders as art_render
 * and also records, before every `every`-th composited sample of a ray
 * (samples every, 2 every, ... K every), the sample's entry distance t, the
 * transmittance T before it and the running sum P = sum of w f (the feature
 * map so far); art_backward_ckpt then splits each ray into K + 1 segments
 * that run in parallel, each starting from its record: the same samples,
 * transmittances and stop as the unsegmented adjoint, with the density
 * gradient's running sum of w (g . f) started at g . P (so only the order of
 * that sum changes).
 *
 * K: records per ray, 1..64; every: samples per segment, 1..65536; rays with
 *    more than (K + 1) every samples run their last segment to the end.
 * ckpt:   device float32 [P][V][H][W][K][C + 4], 8-byte aligned: record j of
 *         a ray = {t as a float64 in words 0-1, T, P[C], one unused word}.
 * ckpt_n: device int32 [P][V][H][W]: records written (min(K, (n - 1) / every)
 *         for a ray of n >= 1 composited samples, else 0); entries of rays in
 *         tiles that no occupied brick covers are not written (the adjoint
 *         does not read them).
 * Both are caller-owned; art_backward_ckpt must get those written by an
 * art_render_ckpt call with the same poses, cameras, FLUT, lambda_th,
 * flags, K and every, together with its out_feat and out_tfinal.
 * Errors: as art_render / art_backward, and ART_EINVAL for K, every, null
 * or misaligned checkpoint buffers.
 */
art_status art_render_ckpt(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                           float lambda_th, unsigned flags,
                           float* out_feat, float* out_alpha, float* out_tfinal,
                           int K, int every, float* ckpt, int32_t* ckpt_n);
art_status art_backward_ckpt(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                             float lambda_th, unsigned flags,
                             const float* out_feat, const float* out_tfinal,
                             const float* d_feat, const float* d_alpha,
                             float* d_sigma, float* d_leaf_feat,
                             int K, int every, const float* ckpt, const int32_t* ckpt_n);

/* ---------------------------------------------------------------------------
 * Learned ray-interval proposal (an addition to the paper's renderer: a small
 * network predicts, per ray, the stretch of the ray that holds its composited
 * samples, so that the traversal can skip the empty part of the ray in front
 * of the surface)
 * ------------------------------------------------------------------------- */

/* Default margin m added on both sides of a proposed interval, in leaf edges h. */
#define ART_PROPOSAL_MARGIN_H 2.0f

/*
 * Training labels of the proposal from the plain renderer: every ray of the
 * current poses x cameras is traversed exactly as by art_render (same
 * arguments and flags) and labels[ray] = (u_near, u_far) receives the entry t
 * of its first and the exit t of its last composited sample, mapped to [0, 1]
 * over the ray's span [t_a, t_b] inside the posed root ([-1, 1]^3, t_a >= 0).
 * Rays with no composited sample (including rays that miss the root) get the
 * empty interval (1, 0).
 * labels: device float32 [P][V][H][W][2].
 * Errors: as art_render.
 */
art_status art_proposal_labels(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                               float lambda_th, unsigned flags, float* labels);

/*
 * Forward render (as art_render) whose traversal starts from a proposed
 * interval per ray.  intervals: device float32 [P][V][H][W][2] of (u_near,
 * u_far) in the units of art_proposal_labels, or NULL to take them from the
 * proposal network (art_proposal_set_weights; evaluated for the rays of every
 * 8x8 tile that holds a brick).  A ray with u_near <= u_far first traverses
 * only [t_a + u_near (t_b - t_a) - m, t_a + u_far (t_b - t_a) + m] clipped to
 * [t_a, t_b], with m = margin_h * h; it falls back to the full traversal of
 * [t_a, t_b] when that interval held no occupied voxel (F1) or, with
 * f2_tau >= 0, when its transmittance on leaving the interval before t_b is
 * still >= f2_tau (F2).  With ART_PROPOSAL_NEAR_ONLY in flags the interval
 * ends at t_b (only the empty front of the ray is skipped; F2 cannot occur).
 * A ray with u_near > u_far (predicted empty) is traversed in full.  The
 * result equals art_render's whenever every skipped part of a ray holds no
 * occupied voxel.
 * Errors: as art_render; ART_EINVAL for a negative or non-finite margin_h or
 * a NaN f2_tau; ART_ESTATE for NULL intervals without network weights.
 */
art_status art_render_proposal(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                               float lambda_th, unsigned flags, const float* intervals, float margin_h,
                               float f2_tau, float* out_feat, float* out_alpha, float* out_tfinal);

/*
 * Forward render (as art_render) that also writes the depth buffer of the
 * hybrid rendering (Section 3.1, paragraph "Hybrid Rendering"): per pixel,
 * the distance along the ray (unit direction, from the camera centre) at
 * which it enters the first occupied posed voxel (its collision winner) whose
 * canonical density, as stored, exceeds depth_sigma (strictly).  The search
 * covers the whole clipped ray: the early stop of the compositing does not
 * end it.  Pixels with no such voxel, including every pixel of an empty
 * tile, get +inf.  out_depth:
 * device float32 [P][V][H][W], written in full.  The feature, opacity and
 * transmittance maps are those of art_render, bit for bit.
 * Errors: as art_render; ART_EINVAL for a NULL out_depth or a NaN depth_sigma.
 */
art_status art_render_depth(art_ctx* ctx, int C, art_dtype dtype, const void* sigma, const void* feat,
                            float lambda_th, unsigned flags, float depth_sigma, float* out_feat, float* out_alpha,
                            float* out_tfinal, float* out_depth);

/*
 * Forward render (as art_render) with view-dependent features: Eq. 5 with
 * S(f, d^c) of Eq. 2 in place of f.  feat: device [n][H][C] (FP32 or BF16 per
 * dtype), H = 1, 4 or 9 real spherical-harmonic coefficients (degrees 0..2,
 * orthonormal, ordered by degree then m = -l..l, no Condon-Shortley phase:
 * Y = 1/(2 sqrt pi); sqrt(3/(4 pi)) (y, z, x); sqrt(15/pi)/2 xy,
 * sqrt(15/pi)/2 yz, sqrt(5/pi)/4 (3z^2 - 1), sqrt(15/pi)/2 xz,
 * sqrt(15/pi)/4 (x^2 - y^2)) of C channels per leaf.  A sample of leaf i
 * contributes w_i sum_h k_{i,h} Y_h(d^c), d^c = R^T d with d the ray's unit
 * direction and R the rotation of the leaf's dominant bone (largest skin
 * weight) in the pose: the reading of the voxel rotation R_i^t.  Outputs as
 * art_render.
 * Errors: as art_render; ART_EUNSUPPORTED for H not in {1, 4, 9} or more than
 * 64 bones.
 */
art_status art_render_sh(art_ctx* ctx, int C, int H, art_dtype dtype, const void* sigma, const void* feat,
                         float lambda_th, unsigned flags, float* out_feat, float* out_alpha, float* out_tfinal);

/*
 * Neural shading network G of Section 3.1 ("Neural Shading"), the "Light"
 * variant of the runtime analysis (Tab. 5): a single encoder-decoder (U-Net)
 * branch that turns the feature map F into RGB and an opacity map, in half
 * precision.  Layers (3x3 convolutions, padding 1, bias, ReLU): encoder levels
 * of 32, 64, 128, 256 channels, two convolutions each, 2x2 max pooling between
 * levels; decoder levels of 128, 64, 32 channels whose first convolution reads
 * the concatenation [encoder output of the level, nearest 2x upsampling of the
 * level below], then a second convolution; a 1x1 head to 4 channels and a
 * sigmoid.  FP16 operands and activations, FP32 accumulation (matrix cores),
 * FP32 head.
 *
 * art_shading_param_count: FP32 parameters for C input channels (1..32), in
 * the order of the 14 convolutions (weight [Cout][Cin][3][3], then bias
 * [Cout]; layer 0 has Cin = C), then the head (weight [4][32], bias [4]);
 * -1 for C outside 1..32.
 * art_shading_set_weights: copy them in (host), converted to FP16.
 * art_shading_forward: N maps F (device float32 [N][C][H][W], H and W
 * multiples of 8) -> out (device float32 [N][4][H][W]: R, G, B, opacity).
 * Enqueued on the context's stream; activations use a context buffer of
 * 332 bytes per pixel of the batch.
 * Errors: ART_EINVAL (counts, NULL, non-finite weights, sizes),
 * ART_EUNSUPPORTED (C), ART_ESTATE (no weights for this C), ART_ENOMEM.
 */
int64_t art_shading_param_count(int C);
art_status art_shading_set_weights(art_ctx* ctx, int C, int64_t count, const float* w);
art_status art_shading_forward(art_ctx* ctx, int C, int N, int H, int W, const float* F, float* out);

/*
 * art_shading_forward for callers that cannot allocate device memory during
 * the call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels, arguments, layouts and results, but the
 * activations live in a fixed array of ART_SHADING_NOALLOC_BYTES that the
 * library holds on every GPU it runs on (from its load until the process
 * ends) instead of a context buffer; the call allocates nothing.  The weights
 * (art_shading_set_weights) and the caller's F and out are used as in
 * art_shading_forward.
 * A batch needs 332 bytes per pixel of N * H * W plus under 3 KB of
 * alignment: at most about 303,000 pixels (one 512 x 512 map, two of
 * 384 x 384).
 * Every call on one GPU, from any context, uses that GPU's one array and
 * leaves the last call's activations in it: calls that overlap on one GPU
 * (other streams, threads or contexts) race, and the caller serialises them.
 * Errors: as art_shading_forward; ART_EINVAL when the batch needs more than
 * ART_SHADING_NOALLOC_BYTES (nothing is enqueued).
 */
#define ART_SHADING_NOALLOC_BYTES 100663296u   /* 96 MiB */
art_status art_shading_forward_noalloc(art_ctx* ctx, int C, int N, int H, int W, const float* F, float* out);

/*
 * Voxel regularisation term of Section 3.1 ("Training", Eq. 10) for every pose
 * and its gradient with respect to the features.  For each canonical leaf i
 * whose posed centre lies inside the posed root, Q(p_i^t, T^t) is the feature
 * of the leaf the posed octree holds at that cell (the collision winner:
 * smallest leaf id); the pose's term is lambda_vrt / N_v * sum_i
 * |Q(p_i^t, T^t) - f_i|_1 with N_v the leaves inside the root, and the terms
 * of all poses add up.  feat: device [n][C] (FP32 or BF16 per dtype).
 * d_feat: device float32 [n][C]; the gradient is ADDED (sign(Q - f_i) *
 * lambda / N_v to the winner's row, its negative to leaf i's), so the buffer
 * can also hold art_backward's gradient.  *loss (host) receives the loss.
 * flags: ART_GEOM_FP32, ART_REUSE_BUILD (use the octrees the last whole-batch
 * render left when they still apply), or 0.
 * Errors: ART_EINVAL (NULL pointer, negative or non-finite lambda_vrt, other
 * flag bits), ART_EUNSUPPORTED (C), ART_ESTATE (missing octree, skin,
 * skeleton or poses).
 */
art_status art_vrt(art_ctx* ctx, int C, art_dtype dtype, const void* feat, float lambda_vrt, unsigned flags,
                   float* d_feat, double* loss);

/*
 * The point-query operator Q of Eq. 10 as an index: for each of n points of
 * the posed space (device float64 [n][3]) of pose `pose`, the canonical leaf
 * the posed octree holds at the point's cell (floor((p + 1) / h) on the posed
 * lattice), or -1 when the cell is empty or outside the posed root.
 * leaf: device int32 [n].
 * Errors: ART_EINVAL (n < 0, NULL with n > 0, pose out of range, unknown
 * flags), ART_ESTATE (missing octree, skin, skeleton or poses).
 */
art_status art_query(art_ctx* ctx, int pose, unsigned flags, int64_t n, const double* points, int32_t* leaf);

/*
 * Map loss of the FLUT training loop (Section 3.1, "Training", with the
 * shading network left out: the rendered maps are compared with target maps
 * directly, reading A23) over R = rays pixels:
 * L = 1/(2R) [sum (F - F*)^2 + sum (A - A*)^2], the A term only when
 * A_target is not NULL.  F, F_target, d_feat: device float32 [n_feat];
 * A, A_target, d_alpha: device float32 [rays].  Writes dL/dF = (F - F*) / R
 * and dL/dA = (A - A*) / R; *loss (host) receives L, summed in FP64 in a
 * fixed order.  Synchronous.
 * Errors: ART_EINVAL (n_feat < 0, rays < 1, a NULL buffer that is needed).
 */
art_status art_map_loss(art_ctx* ctx, int64_t n_feat, int64_t rays, const float* F, const float* F_target,
                        const float* A, const float* A_target, float* d_feat, float* d_alpha, double* loss);

/*
 * One Adam update (step counts from 1, bias-corrected) of a device float32
 * FLUT array of `count` entries from its gradient, moments m and v updated in
 * place, then param = max(param, lower) (pass -INFINITY for none; 0 keeps
 * densities non-negative).  Enqueued on the context's stream.
 * Errors: ART_EINVAL (count < 0, NULL buffer, step < 1, lr < 0, beta outside
 * [0, 1), eps <= 0, NaN lower).
 */
art_status art_flut_adam(art_ctx* ctx, int64_t count, float* param, const float* grad, float* m, float* v, int step,
                         float lr, float beta1, float beta2, float eps, float lower);

/*
 * The proposal network: x = [o (3), d (3), pose code (6 J)] -> 64 -> 64 -> 64
 * (ReLU) -> 2 (sigmoid) = (u_near, u_far), where (o, d) is the ray (origin,
 * unit direction, FP32) and the pose code holds, per bone j, the first and
 * second column of the rotation of its axis-angle r_j.  Matrix products use
 * BF16 operands with FP32 accumulation; the pose-code part of the first layer
 * is evaluated per pose in FP32.  Weights are FP32, flat in the order W1
 * [64][6 + 6J], b1 [64], W2 [64][64], b2, W3 [64][64], b3, W4 [2][64], b4 [2]
 * (row-major [out][in]).
 * Returns the parameter count for J bones (24258 for J = 40), -1 for J
 * outside 1..255.
 */
int64_t art_proposal_param_count(int J);

/* Copy `count` host FP32 weights in (resets the Adam state) / out.
 * Errors: ART_ESTATE (no skeleton; get: no weights for the current skeleton),
 * ART_EINVAL (count mismatch, NULL, non-finite weight). */
art_status art_proposal_set_weights(art_ctx* ctx, int64_t count, const float* w);
art_status art_proposal_get_weights(art_ctx* ctx, int64_t count, float* w);

/* Seeded initial weights (resets the Adam state, as art_proposal_set_weights):
 * every weight and bias of a layer with fan-in m is (2u - 1) / sqrt(m), u in
 * [0, 1) the top 24 bits of output i + 1 of the SplitMix64 stream of `seed`
 * (Steele, Lea and Flood, OOPSLA 2014) for flat parameter index i (the order
 * of art_proposal_set_weights).  The same seed gives the same weights on any
 * device.
 * Errors: ART_ESTATE (no skeleton). */
art_status art_proposal_init(art_ctx* ctx, uint64_t seed);

/*
 * Network inputs and targets of selected rays: ray_id (device int64 [n]) are
 * indices into [P][V][H][W] of the current poses and cameras; labels is the
 * device output of art_proposal_labels.  Writes od (device float32 [n][6]: the
 * ray origin and direction in FP32), pose (device int32 [n]) and target
 * (device float32 [n][2]).  Synchronous.
 * Errors: ART_ESTATE (no poses or cameras), ART_EINVAL (NULL, an id out of
 * range).
 */
art_status art_proposal_gather(art_ctx* ctx, int64_t n, const int64_t* ray_id, const float* labels, float* od,
                               int32_t* pose, float* target);

/*
 * Network outputs for n rays: od (device float32 [n][6]), pose (device int32
 * [n], indices of the current poses) -> out (device float32 [n][2]).
 * Synchronous.  Errors: ART_ESTATE (no weights for the current skeleton, no
 * poses), ART_EINVAL (NULL, n < 0, a pose id out of range).
 */
art_status art_proposal_forward(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, float* out);

/*
 * Training loss of the network (a context setting, used by
 * art_proposal_grad and art_proposal_train): kind 0, SmoothL1 with beta = 1
 * on both outputs (the default); kind 1, one-sided: on rays whose label holds
 * a sample (u_near <= u_far) the pinball (quantile) loss
 * rho_tau(t - y) = max(tau (t - y), (tau - 1) (t - y)) of target t and output y
 * at level tau_near for u_near and tau_far for u_far, and SmoothL1 on rays with
 * the empty label (1, 0), which keeps them predicted empty.  Minimised over a
 * constant, the pinball loss gives the tau-quantile of the targets: a small
 * tau_near makes late starts rare, a large tau_far early ends.
 * Errors: ART_EINVAL (kind not 0 or 1; kind 1 with a level outside (0, 1)).
 */
art_status art_proposal_set_loss(art_ctx* ctx, int kind, float tau_near, float tau_far);

/*
 * Loss L = mean over the n rays and both outputs of the training loss
 * (art_proposal_set_loss; SmoothL1 by default) between the network outputs
 * and target (device float32 [n][2]), and its
 * gradient with respect to the weights: grad (device float32 [count]), loss
 * (device float32 [1]).  The weight gradients are contractions over rays on
 * the matrix cores (BF16 operands, the deltas stored in BF16); partial sums
 * over chunks of rays are added in a fixed order, so the result is
 * deterministic.  n in 1..2^20.  Synchronous.
 * Errors: as art_proposal_forward.
 */
art_status art_proposal_grad(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, const float* target,
                             float* grad, float* loss);

/*
 * `steps` Adam steps (bias-corrected) on the FP32 weights, step s on the rays
 * [(s mod (n / batch)) * batch, + batch) of the device arrays od / pose /
 * target (shuffle them beforehand; n mod batch rays at the end are unused).
 * The Adam state persists across calls until the weights are set again.
 * loss_log: host float32 [steps] of the batch losses (before each update), or
 * NULL.  batch in 1..2^20, n >= batch.  Synchronous.
 * Errors: as art_proposal_forward; ART_EINVAL for hyper-parameters outside
 * lr > 0, 0 <= beta < 1, eps > 0.
 */
art_status art_proposal_train(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, const float* target,
                              int64_t batch, int steps, float lr, float beta1, float beta2, float eps,
                              float* loss_log);

/*
 * Start margin of the guided traversal for the current network, from
 * held-out rays (the arrays of art_proposal_gather): for each ray whose label
 * holds a sample (u_near <= u_far), its late start in leaf edges h,
 * (predicted u_near - labelled u_near) * (t_b - t_a) / h with [t_a, t_b] the
 * ray's span inside the posed root ([-1, 1]^3, t_a >= 0); *margin_h (host)
 * receives the `quantile` of these values (linear interpolation between
 * order statistics), at least floor_h; floor_h when no ray has a sample.
 * A margin at the 0.999 quantile covers all but 0.1 % of the late starts on
 * the held-out rays.  Synchronous.
 * Errors: as art_proposal_forward; ART_EINVAL for quantile outside [0, 1] or
 * a negative or non-finite floor_h.
 */
art_status art_proposal_calibrate(art_ctx* ctx, int64_t n, const float* od, const int32_t* pose, const float* target,
                                  float quantile, float floor_h, float* margin_h);

/*
 * Save (save != 0) or load the proposal network's training state: the FP32
 * weights, both Adam moments and the Adam step count, so that training
 * resumes where it stopped (the next art_proposal_train step continues the
 * bias correction from the saved count and gives the same weights, bit for
 * bit, as an uninterrupted run).  File (little-endian): the 8 bytes
 * "ARTPROP1", int32 J, int32 0, int64 parameter count, int64 step, then the
 * weights, the first and the second moments (FP32, the order of
 * art_proposal_set_weights).  Loading checks the magic, J, the count, that
 * every value is finite and the second moments are >= 0, and that nothing
 * follows; on failure the context keeps its previous state.  Synchronous.
 * Errors: ART_EINVAL (NULL path, I/O failure, a file that does not match),
 * ART_ESTATE (no skeleton; save: no weights for the current skeleton).
 */
art_status art_proposal_io(art_ctx* ctx, int save, const char* path);

/* ---------------------------------------------------------------------------
 * Inspection of intermediate results (parity tests, debugging)
 * ------------------------------------------------------------------------- */

/*
 * Skinning matrices B_j = M^t_j (M^c_j)^-1 of Eq. 4 as composed on the GPU in
 * FP64: B: host float64 [P][J][3][4].  Synchronous.
 */
art_status art_get_bones(art_ctx* ctx, double* B);

/*
 * Posed Morton key of every canonical leaf for pose `pose` (0xFFFFFFFF for a
 * dropped leaf).  keys: device uint32 [n].  flags: ART_GEOM_FP32 or 0.
 * Synchronous.
 */
art_status art_get_posed_keys(art_ctx* ctx, int pose, unsigned flags, uint32_t* keys);

/*
 * Posed octree of pose `pose`: the occupied cells in Morton order with their
 * collision winners, and the level of 8^3-leaf bricks.
 * counts: host int64 [4] = {M occupied cells, nb bricks, dropped leaves,
 *         collisions (= n - dropped - M)}.
 * keys, winner: device uint32 [n] (first M valid);
 * brick_keys (key >> 9), brick_row (index of the brick's first cell in keys):
 *         device uint32 [n] (first nb valid);
 * brick_mask: device uint32 [n][16] (first nb valid), bit (key & 511) set for
 *         each occupied cell of the brick.
 * Any of the device pointers may be NULL.  Synchronous.
 */
art_status art_get_octree(art_ctx* ctx, int pose, unsigned flags, int64_t* counts,
                          uint32_t* keys, uint32_t* winner, uint32_t* brick_keys,
                          uint32_t* brick_row, uint32_t* brick_mask);

/*
 * Composited samples of every ray of (pose, view), in front-to-back order,
 * from the same traversal as art_render: leaf: device int32 [H*W][max_hits]
 * (canonical winner leaf ids), delta: device float64 [H*W][max_hits] (chord
 * lengths), count: device int32 [H*W] (may exceed max_hits; the list is then
 * truncated).  Synchronous.
 */
art_status art_get_hits(art_ctx* ctx, int pose, int view, int C, art_dtype dtype,
                        const void* sigma, const void* feat, float lambda_th, unsigned flags,
                        int max_hits, int32_t* leaf, double* delta, int32_t* count);

/*
 * Outcome of the last render / backward call made with ART_ASYNC: synchronises
 * the context's stream, then *overflowed_items receives the number of
 * (pose, view group) items whose tile lists overflowed (their maps were not
 * rendered: render them again, the next call has the capacity) and
 * *bad_densities the number of negative or non-finite FLUT densities (the
 * call rendered nothing); art_get_stats then holds that call's counters.
 * When both are 0 the posed octrees and tile lists the call built may be
 * reused by a following ART_REUSE_BUILD call, as after a synchronous one (an
 * asynchronous call whose status is never read leaves nothing to reuse).
 * Both 0 when the last call was synchronous (it reported such errors itself).
 * Either pointer may be NULL.  Call it before the next render call on the
 * context, which starts a new record.
 * Errors: ART_EINVAL (NULL ctx), ART_EDEVICE.
 */
art_status art_render_status(art_ctx* ctx, int64_t* overflowed_items, int64_t* bad_densities);

/*
 * Counters of the last render / backward / label call, host int64
 * [ART_NUM_STATS]:
 * {rays, composited samples, rays with at least one sample, dropped leaves,
 *  collisions, bricks (summed over poses), tile/brick pairs, kernel launches,
 *  tile-list entries summed over the 8x8 tiles, traversal rounds summed over
 *  the compositing kernel's waves, ray/voxel partition steps summed over rays,
 *  rays of the tiles the compositing kernel rendered (non-empty brick list),
 *  rays that started from a proposed interval, rays of those that fell back
 *  to the full traversal (art_render_proposal only; 0 otherwise),
 *  leaf-gradient additions (art_backward only: one per composited sample, or
 *  one per distinct leaf of a burst when the adjoint merges them; 0 otherwise)}.
 */
#define ART_NUM_STATS 15
art_status art_get_stats(art_ctx* ctx, int64_t* stats);

/*
 * Per-stage GPU time of the last call made with ART_TIMING, host float [7] in
 * milliseconds: {fk, skin, octree build, tile binning, render, total,
 * proposal-network inference}, summed over poses.  `render` covers only the
 * compositing kernel launches; n_render receives their number.
 */
art_status art_get_timing(art_ctx* ctx, float* ms, int* n_render);

#ifdef __cplusplus
}
#endif

#endif /* ARTEMIS_H */
