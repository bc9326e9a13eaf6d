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
                            const PoseCounters* __restrict__ cnt, BinGeom g,
                            uint32_t* __restrict__ out) {
    const uint32_t total = cnt->nb * (uint32_t)g.Vg;
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
                           PoseCounters* __restrict__ cnt, BinGeom g,
                           const uint32_t* __restrict__ off, uint32_t* __restrict__ pk,
                           uint32_t* __restrict__ pv) {
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

__global__ void k_tile_mark(const uint32_t* __restrict__ pk, const PoseCounters* __restrict__ cnt,
                            int mbits, uint32_t* __restrict__ tstart, uint32_t* __restrict__ tend) {
    const uint32_t n = cnt->pad[0];
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

__global__ void k_bin_items(PoseCounters* __restrict__ cnt, uint32_t Vg) {
    cnt->pad[1] = cnt->nb * Vg;
}

// count -> scan -> emit -> stable sort -> per-tile ranges.  The sorted brick
// ids end in pair_out; the sort ping-pongs between the scratch buffer and
// pair_out so that its last pass writes pair_out.
hipError_t launch_bin(Scratch& s, const CamParams* cam_dev, const uint32_t* brick_key, int v0, int Vg,
                      int H, int W, int depth, bool fp32, uint32_t* pair_out, uint32_t* tile_start,
                      uint32_t* tile_end, hipStream_t st, int* launches) {
    BinGeom g = make_geom(s, v0, Vg, H, W, depth);
    const int key_bits = bits_for((uint64_t)Vg * g.TPV - 1) + g.mbits;
    const int passes = (key_bits + 7) / 8;
    PoseCounters* cnt = s.counters.as<PoseCounters>();
    hipLaunchKernelGGL(k_bin_items, dim3(1), dim3(1), 0, st, cnt, (uint32_t)Vg);
    hipLaunchKernelGGL(k_bin_count, dim3(2048), dim3(256), 0, st, cam_dev, brick_key,
                       (const PoseCounters*)cnt, g, s.bin_cnt.as<uint32_t>());
    *launches += 2;
    hipError_t e = launch_scan_exclusive(s.bin_cnt.as<uint32_t>(), s.bin_off.as<uint32_t>(),
                                         &cnt->pad[1], &cnt->npairs, s.blk0.as<uint32_t>(), st,
                                         launches);
    if (e != hipSuccess) return e;
    // an even number of passes ends where it starts
    uint32_t* v_first = (passes & 1) ? s.pv0.as<uint32_t>() : pair_out;
    uint32_t* v_second = (passes & 1) ? pair_out : s.pv0.as<uint32_t>();
    if (fp32)
        hipLaunchKernelGGL(k_bin_emit<float>, dim3(2048), dim3(256), 0, st, cam_dev, brick_key, cnt, g,
                           s.bin_off.as<uint32_t>(), s.pk0.as<uint32_t>(), v_first);
    else
        hipLaunchKernelGGL(k_bin_emit<double>, dim3(2048), dim3(256), 0, st, cam_dev, brick_key, cnt, g,
                           s.bin_off.as<uint32_t>(), s.pk0.as<uint32_t>(), v_first);
    *launches += 1;
    bool in1 = false;
    e = launch_radix_sort(s.pk0.as<uint32_t>(), v_first, s.pk1.as<uint32_t>(), v_second, &cnt->pad[0],
                          (uint32_t)s.pair_cap, key_bits, s.hist.as<uint32_t>(),
                          s.digit_tot.as<uint32_t>(), st, &in1, launches);
    if (e != hipSuccess) return e;
    const uint32_t* pk = in1 ? s.pk1.as<uint32_t>() : s.pk0.as<uint32_t>();
    const size_t tiles = (size_t)Vg * g.TPV;
    e = launch_fill_u32(tile_start, 0u, tiles, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(tile_end, 0u, tiles, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_mark, dim3(2048), dim3(256), 0, st, pk, (const PoseCounters*)cnt, g.mbits,
                       tile_start, tile_end);
    *launches += 3;
    return hipGetLastError();
}

}  // namespace art
