// Per-tile brick lists for ray indexing (Section 3.1: rays are tested only
// against the voxels of the rebuilt octree).
//
// Each 8x8-pixel tile of each view gets the list of occupied bricks whose
// screen-space bounding box covers one of its pixel centres, sorted front to
// back.  The order key of a brick is its Manhattan distance, in bricks, from
// the brick holding the camera centre: along any ray leaving the camera every
// brick step moves one (or more) coordinates one brick further from that
// brick, so the key grows strictly along every ray, and a list sorted by it
// visits every ray's bricks in increasing t.  Bricks with equal keys are never
// crossed by the same ray, so their relative order does not matter.
//
//   k_bin_count : per (brick, view) number of covered tiles
//   (exclusive scan)
//   k_bin_emit  : per (brick, view) one (tile << mbits | order key, brick) pair
//                 per covered tile
//   (stable radix sort of the pairs)
//   k_tile_mark : first / one-past-last pair of each tile
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace art {

struct BinGeom {
    int v0, Vg, H, W, TX, TY, TPV, GB, mbits;
    double h;
    uint32_t cap;
};

__device__ inline void brick_coords(uint32_t bkey, int* bx, int* by, int* bz) {
    *bx = (int)compact3(bkey);
    *by = (int)compact3(bkey >> 1);
    *bz = (int)compact3(bkey >> 2);
}

// Covered tile rectangle of brick b in view v; returns false if none.
__device__ inline bool brick_tile_rect(const CamParams& c, int bx, int by, int bz,
                                       const BinGeom& g, int* tx0, int* tx1, int* ty0, int* ty1) {
    const double s = 8.0 * g.h;
    const double lo[3] = {fmax(-1.0, -1.0 + bx * s), fmax(-1.0, -1.0 + by * s), fmax(-1.0, -1.0 + bz * s)};
    const double hi[3] = {fmin(1.0, -1.0 + (bx + 1) * s), fmin(1.0, -1.0 + (by + 1) * s),
                          fmin(1.0, -1.0 + (bz + 1) * s)};
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    bool behind = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double X = ((q & 1) ? hi[0] : lo[0]) - c.t[0];
        const double Y = ((q & 2) ? hi[1] : lo[1]) - c.t[1];
        const double Z = ((q & 4) ? hi[2] : lo[2]) - c.t[2];
        // camera coordinates: columns of R are the camera axes
        const double xc = c.R[0] * X + c.R[3] * Y + c.R[6] * Z;
        const double yc = c.R[1] * X + c.R[4] * Y + c.R[7] * Z;
        const double zc = c.R[2] * X + c.R[5] * Y + c.R[8] * Z;
        if (zc <= 1e-9) {
            behind = true;
        } else {
            const double u = c.fx * xc / zc + c.cx;
            const double v = c.fy * yc / zc + c.cy;
            umin = fmin(umin, u);
            umax = fmax(umax, u);
            vmin = fmin(vmin, v);
            vmax = fmax(vmax, v);
        }
    }
    if (behind) {   // a corner at or behind the camera plane: every tile (conservative)
        *tx0 = 0; *tx1 = g.TX - 1; *ty0 = 0; *ty1 = g.TY - 1;
        return true;
    }
    const double m = 0.01;   // pixels of safety margin for rounding
    const double fx0 = ceil(umin - m - 0.5), fx1 = floor(umax + m - 0.5);
    const double fy0 = ceil(vmin - m - 0.5), fy1 = floor(vmax + m - 0.5);
    if (fx1 < 0.0 || fy1 < 0.0 || fx0 > g.W - 1 || fy0 > g.H - 1 || fx0 > fx1 || fy0 > fy1)
        return false;
    const int x0 = (int)fmax(fx0, 0.0), x1 = (int)fmin(fx1, (double)(g.W - 1));
    const int y0 = (int)fmax(fy0, 0.0), y1 = (int)fmin(fy1, (double)(g.H - 1));
    *tx0 = x0 >> 3; *tx1 = x1 >> 3; *ty0 = y0 >> 3; *ty1 = y1 >> 3;
    return true;
}

// Brick of the camera centre as the traversal sees the ray origin (precision R),
// clamped to one brick outside the grid.
template <typename R>
__device__ inline void eye_brick(const CamParams& c, const BinGeom& g, int* e) {
    const R invh = (R)(1.0 / g.h);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R q = (R)1 + (R)c.t[a];
        const R u = floor(q * invh);
        R eb = floor(u / (R)8);
        if (eb < (R)-1) eb = (R)-1;
        if (eb > (R)g.GB) eb = (R)g.GB;
        e[a] = (int)eb;
    }
}

__global__ void k_bin_count(const CamParams* __restrict__ cam, const uint32_t* __restrict__ brick_key,
                            size_t key_stride, const PoseCounters* __restrict__ cnt, BinGeom g,
                            uint32_t* __restrict__ out, size_t out_stride) {
    brick_key += blockIdx.y * key_stride;
    out += blockIdx.y * out_stride;
    const uint32_t total = cnt[blockIdx.y].nb * (uint32_t)g.Vg;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint32_t b = i / g.Vg;
        const int v = g.v0 + (int)(i % g.Vg);
        int bx, by, bz, tx0, tx1, ty0, ty1;
        brick_coords(brick_key[b], &bx, &by, &bz);
        uint32_t n = 0;
        if (brick_tile_rect(cam[v], bx, by, bz, g, &tx0, &tx1, &ty0, &ty1))
            n = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
        out[i] = n;
    }
}

template <typename R>
__global__ void k_bin_emit(const CamParams* __restrict__ cam, const uint32_t* __restrict__ brick_key,
                           size_t key_stride, PoseCounters* __restrict__ cnt, BinGeom g,
                           const uint32_t* __restrict__ off, size_t off_stride, uint32_t* __restrict__ pk,
                           size_t pk_stride, uint32_t* __restrict__ pv, size_t pv_stride) {
    brick_key += blockIdx.y * key_stride;
    cnt += blockIdx.y;
    off += blockIdx.y * off_stride;
    pk += blockIdx.y * pk_stride;
    pv += blockIdx.y * pv_stride;
    const uint32_t total = cnt->nb * (uint32_t)g.Vg;
    const uint32_t npairs = cnt->npairs;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cnt->overflow = npairs > g.cap ? 1u : 0u;
        cnt->pad[0] = npairs > g.cap ? g.cap : npairs;   // number of pairs to sort
    }
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint32_t b = i / g.Vg;
        const int vv = (int)(i % g.Vg);
        const int v = g.v0 + vv;
        int bx, by, bz, tx0, tx1, ty0, ty1;
        brick_coords(brick_key[b], &bx, &by, &bz);
        if (!brick_tile_rect(cam[v], bx, by, bz, g, &tx0, &tx1, &ty0, &ty1)) continue;
        int e[3];
        eye_brick<R>(cam[v], g, e);
        const uint32_t mkey = (uint32_t)(abs(bx - e[0]) + abs(by - e[1]) + abs(bz - e[2]));
        uint32_t o = off[i];
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx, ++o) {
                if (o >= g.cap) continue;
                const uint32_t tile = (uint32_t)(vv * g.TPV + ty * g.TX + tx);
                pk[o] = (tile << g.mbits) | mkey;
                pv[o] = b;
            }
    }
}

__global__ void k_tile_mark(const uint32_t* __restrict__ pk, size_t pk_stride,
                            const PoseCounters* __restrict__ cnt, int mbits, uint32_t* __restrict__ tstart,
                            uint32_t* __restrict__ tend, size_t t_stride) {
    pk += blockIdx.y * pk_stride;
    tstart += blockIdx.y * t_stride;
    tend += blockIdx.y * t_stride;
    const uint32_t n = cnt[blockIdx.y].pad[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t t = pk[i] >> mbits;
        if (i == 0 || (pk[i - 1] >> mbits) != t) tstart[t] = i;
        if (i + 1 == n || (pk[i + 1] >> mbits) != t) tend[t] = i + 1;
    }
}

static int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 32 && (1ull << b) <= maxval) ++b;
    return b;
}

static BinGeom make_geom(const Scratch& s, int v0, int Vg, int H, int W, int depth) {
    BinGeom g;
    g.v0 = v0;
    g.Vg = Vg;
    g.H = H;
    g.W = W;
    g.TX = (W + 7) / 8;
    g.TY = (H + 7) / 8;
    g.TPV = g.TX * g.TY;
    const int G = 2 << depth;
    g.GB = G >= 8 ? G / 8 : 1;
    g.mbits = bits_for((uint64_t)3 * (g.GB + 1));
    g.h = 1.0 / (double)(1 << depth);
    g.cap = (uint32_t)s.pair_cap;
    return g;
}

int bin_key_bits(int Vg, int H, int W, int depth, int* mbits) {
    Scratch dummy;
    BinGeom g = make_geom(dummy, 0, Vg, H, W, depth);
    *mbits = g.mbits;
    return bits_for((uint64_t)Vg * g.TPV - 1) + g.mbits;
}

__global__ void k_bin_items(PoseCounters* __restrict__ cnt, uint32_t Vg, int batch) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < batch) cnt[p].pad[1] = cnt[p].nb * Vg;
}

// Pair counts of a view group for the host: overflow flag and pair count per
// pose (a pose outside `redo`, when given, is marked done so the compositing
// kernel skips it).
__global__ void k_pairs(const PoseCounters* __restrict__ c, unsigned long long* __restrict__ st,
                        uint32_t* __restrict__ ovf, int ngroups, int group, const uint8_t* __restrict__ redo,
                        int batch) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= batch) return;
    const size_t slot = (size_t)p * ngroups + group;
    if (redo && !redo[slot]) {
        ovf[2 * slot] = 1u;
        ovf[2 * slot + 1] = 0u;
        return;
    }
    atomicAdd(&st[6], (unsigned long long)c[p].npairs);
    ovf[2 * slot] = c[p].overflow;
    ovf[2 * slot + 1] = c[p].npairs;
}

// count -> scan -> emit -> stable sort -> per-tile ranges for one view group
// of every pose in the batch.  The sort ping-pongs between the scratch payload
// buffer and the persistent tile lists so that its last pass writes the lists.
hipError_t launch_bin(Scratch& s, const CamParams* cam_dev, const OctreeSlot& o, size_t n, int batch, int V, int v0,
                      int Vg, int group, int ngroups, int H, int W, int depth, bool fp32, hipStream_t st,
                      int* launches) {
    BinGeom g = make_geom(s, v0, Vg, H, W, depth);
    const int key_bits = bits_for((uint64_t)Vg * g.TPV - 1) + g.mbits;
    const int passes = (key_bits + 7) / 8;
    PoseCounters* cnt = s.counters.as<PoseCounters>();
    hipLaunchKernelGGL(k_bin_items, dim3((batch + 63) / 64), dim3(64), 0, st, cnt, (uint32_t)Vg, batch);
    hipLaunchKernelGGL(k_bin_count, dim3(256, batch), dim3(256), 0, st, cam_dev, o.brick_key, n,
                       (const PoseCounters*)cnt, g, s.bin_cnt.as<uint32_t>(), s.bin_stride);
    *launches += 2;
    hipError_t e = launch_scan_exclusive(s.bin_cnt.as<uint32_t>(), s.bin_off.as<uint32_t>(), s.bin_stride,
                                         &cnt[0].pad[1], sizeof(PoseCounters) / 4, &cnt[0].npairs,
                                         sizeof(PoseCounters) / 4, s.blk0.as<uint32_t>(), batch, st, launches);
    if (e != hipSuccess) return e;
    const size_t vstride = (size_t)ngroups * s.pair_cap;
    uint32_t* lists = s.pair_v.as<uint32_t>() + (size_t)group * s.pair_cap;
    uint32_t* scratch = s.pv0.as<uint32_t>() + (size_t)group * s.pair_cap;
    // an even number of passes ends where it starts
    uint32_t* v_first = (passes & 1) ? scratch : lists;
    uint32_t* v_second = (passes & 1) ? lists : scratch;
    if (fp32)
        hipLaunchKernelGGL(k_bin_emit<float>, dim3(256, batch), dim3(256), 0, st, cam_dev, o.brick_key, n, cnt, g,
                           s.bin_off.as<uint32_t>(), s.bin_stride, s.pk0.as<uint32_t>(), s.pair_cap, v_first, vstride);
    else
        hipLaunchKernelGGL(k_bin_emit<double>, dim3(256, batch), dim3(256), 0, st, cam_dev, o.brick_key, n, cnt, g,
                           s.bin_off.as<uint32_t>(), s.bin_stride, s.pk0.as<uint32_t>(), s.pair_cap, v_first, vstride);
    *launches += 1;
    SortBatch sb;
    sb.k0 = s.pk0.as<uint32_t>();
    sb.k1 = s.pk1.as<uint32_t>();
    sb.kstride = s.pair_cap;
    sb.v0 = v_first;
    sb.v1 = v_second;
    sb.vstride = vstride;
    sb.d_n = &cnt[0].pad[0];
    sb.nstride = sizeof(PoseCounters) / 4;
    // size the sort grid by the largest list seen so far (plus a quarter), so
    // that blocks take whole 4096-key tiles; any larger list is still sorted in
    // full (blocks then take several tiles)
    sb.n_cap = (uint32_t)(s.pair_hint ? std::min(s.pair_cap, s.pair_hint + s.pair_hint / 4 + 4096) : s.pair_cap);
    sb.hist = s.hist.as<uint32_t>();
    sb.digit_tot = s.digit_tot.as<uint32_t>();
    sb.batch = batch;
    bool in1 = false;
    e = launch_radix_sort(sb, key_bits, st, &in1, launches);
    if (e != hipSuccess) return e;
    const uint32_t* pk = in1 ? s.pk1.as<uint32_t>() : s.pk0.as<uint32_t>();
    const size_t TPVg = (size_t)V * g.TPV;   // tile stride per pose
    hipLaunchKernelGGL(k_tile_mark, dim3(256, batch), dim3(256), 0, st, pk, s.pair_cap, (const PoseCounters*)cnt,
                       g.mbits, s.tile_start.as<uint32_t>() + (size_t)v0 * g.TPV,
                       s.tile_end.as<uint32_t>() + (size_t)v0 * g.TPV, TPVg);
    *launches += 1;
    return hipGetLastError();
}

}  // namespace art
