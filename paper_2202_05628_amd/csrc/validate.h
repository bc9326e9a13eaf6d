// Host-side checks and conversions of the ABI's inputs (plain C++, no HIP):
// the canonical octree, skin weights, skeleton, poses and cameras.  Each
// function returns "" when the input is valid, else the message the call
// reports with ART_EINVAL.  Kept free of device code so that a sanitizer
// build on the host can exercise them.
#pragma once

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace art {

// Per-view camera as used by the kernels (FP64).
struct CamParams {
    double fx, fy, cx, cy;
    double R[9];   // row-major camera-to-world rotation (columns: right, down, forward)
    double t[3];   // camera centre
};

// Canonical leaves: depth 1..9, 1 <= n <= 8^depth (and < 2^31), every cell
// inside the 2^depth grid, no cell twice.  ijk: [3][n] SoA planes.
inline std::string check_octree(int depth, int64_t n, const uint16_t* ijk) {
    if (depth < 1 || depth > 9) return "depth must be in 1..9";
    if (n < 1 || n > ((int64_t)1 << (3 * depth)) || n > 0x7FFFFFFFLL) return "leaf count out of range";
    if (!ijk) return "ijk is NULL";
    const int64_t G = (int64_t)1 << depth;
    std::vector<uint32_t> lin((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t x = ijk[i], y = ijk[n + i], z = ijk[2 * n + i];
        if (x >= G || y >= G || z >= G) return "leaf " + std::to_string(i) + " outside the 2^depth grid";
        lin[(size_t)i] = (uint32_t)((z * G + y) * G + x);
    }
    std::sort(lin.begin(), lin.end());
    for (size_t i = 1; i < lin.size(); ++i)
        if (lin[i] == lin[i - 1]) return "duplicate leaf cells";
    return "";
}

// Skin weights of n leaves: bone [4][n], weight [4][n] finite and >= 0.
// Outputs the largest bone id and, per leaf, the bone of its largest weight
// (the first of equal ones).
inline std::string check_skin(int64_t n, const uint8_t* bone, const float* weight, int* max_bone,
                              std::vector<uint8_t>* dom) {
    if (!bone || !weight) return "bone / weight is NULL";
    const size_t m = (size_t)n;
    int mb = -1;
    for (size_t i = 0; i < 4 * m; ++i) {
        if (!(weight[i] >= 0.0f) || !std::isfinite(weight[i])) return "skin weights must be finite and >= 0";
        mb = std::max(mb, (int)bone[i]);
    }
    dom->assign(m, 0);
    for (size_t i = 0; i < m; ++i) {
        int best = 0;
        for (int k = 1; k < 4; ++k)
            if (weight[k * m + i] > weight[best * m + i]) best = k;
        (*dom)[i] = bone[best * m + i];
    }
    *max_bone = mb;
    return "";
}

// Skeleton: 1 <= J <= 255, parent[0] = -1, 0 <= parent[j] < j, finite joints.
inline std::string check_skeleton(int J, const int32_t* parent, const double* rest_joint) {
    if (J < 1 || J > 255) return "J must be in 1..255";
    if (!parent || !rest_joint) return "parent / rest_joint is NULL";
    if (parent[0] != -1) return "parent[0] must be -1";
    for (int j = 1; j < J; ++j)
        if (parent[j] < 0 || parent[j] >= j) return "parent[j] must be in [0, j)";
    for (int i = 0; i < 3 * J; ++i)
        if (!std::isfinite(rest_joint[i])) return "rest joints must be finite";
    return "";
}

// P poses of J joints, packed per pose as [r_0 .. r_{J-1}, R, T] (3 doubles each).
inline std::string pack_poses(int J, int P, const double* r, const double* R, const double* T,
                              std::vector<double>* buf) {
    if (P < 1 || P > 4096) return "P must be in 1..4096";
    if (!r || !R || !T) return "r / R / T is NULL";
    buf->assign((size_t)P * (J + 2) * 3, 0.0);
    for (int p = 0; p < P; ++p) {
        double* dst = buf->data() + (size_t)p * (J + 2) * 3;
        memcpy(dst, r + (size_t)p * J * 3, sizeof(double) * J * 3);
        memcpy(dst + J * 3, R + 3 * p, sizeof(double) * 3);
        memcpy(dst + J * 3 + 3, T + 3 * p, sizeof(double) * 3);
    }
    for (double v : *buf)
        if (!std::isfinite(v)) return "pose parameters must be finite";
    return "";
}

// V pinhole cameras (K [V][3][3], c2w [V][3][4]) at H x W: finite values,
// non-zero focal lengths, an orthonormal rotation.
inline std::string check_cameras(int V, int H, int W, const double* K, const double* c2w,
                                 std::vector<CamParams>* cams) {
    if (V < 1 || V > 4096) return "V must be in 1..4096";
    if (H < 1 || H > 8192 || W < 1 || W > 8192) return "H, W must be in 1..8192";
    if (!K || !c2w) return "K / c2w is NULL";
    cams->assign((size_t)V, CamParams{});
    for (int v = 0; v < V; ++v) {
        const double* k = K + 9 * v;
        const double* m = c2w + 12 * v;
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(k[i])) return "K must be finite";
        for (int i = 0; i < 12; ++i)
            if (!std::isfinite(m[i])) return "c2w must be finite";
        if (!(k[0] != 0.0) || !(k[4] != 0.0)) return "focal lengths must be non-zero";
        // the camera-to-world rotation must be orthonormal (columns: right, down, forward)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double dot = 0.0;
                for (int r = 0; r < 3; ++r) dot += m[4 * r + a] * m[4 * r + b];
                if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-6) return "c2w rotation must be orthonormal";
            }
        CamParams& c = (*cams)[(size_t)v];
        c.fx = k[0];
        c.fy = k[4];
        c.cx = k[2];
        c.cy = k[5];
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) c.R[3 * a + b] = m[4 * a + b];
            c.t[a] = m[4 * a + 3];
        }
    }
    return "";
}

}  // namespace art
