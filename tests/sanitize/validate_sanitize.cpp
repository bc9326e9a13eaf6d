// Host sanitizer driver of the ABI's input checks (csrc/validate.h): built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  Valid inputs at the edges of every range are
// accepted and each kind of invalid input is refused with a message; the
// conversions (pose packing, camera parameters, dominant bones) are checked
// value by value.  Exit status 0 when every check passes.
#include <cmath>
#include <cstdio>
#include <limits>
#include <vector>

#include "validate.h"

using namespace art;

static int fails = 0;
static void ok(bool c, const char* what) {
    if (!c) {
        std::fprintf(stderr, "check failed: %s\n", what);
        ++fails;
    }
}

int main() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    // ---- octree -------------------------------------------------------------------
    {
        // every cell of a 2^1 grid (n = 8 = 8^depth, the largest count)
        std::vector<uint16_t> ijk(24);
        for (int i = 0; i < 8; ++i) {
            ijk[i] = i & 1;
            ijk[8 + i] = (i >> 1) & 1;
            ijk[16 + i] = i >> 2;
        }
        ok(check_octree(1, 8, ijk.data()).empty(), "full depth-1 grid accepted");
        ok(!check_octree(0, 8, ijk.data()).empty(), "depth 0 refused");
        ok(!check_octree(10, 8, ijk.data()).empty(), "depth 10 refused");
        ok(!check_octree(1, 9, ijk.data()).empty(), "more leaves than cells refused");
        ok(!check_octree(1, 0, ijk.data()).empty(), "no leaves refused");
        ok(!check_octree(1, 8, nullptr).empty(), "NULL refused");
        std::vector<uint16_t> dup = ijk;
        dup[7] = 0;
        dup[15] = 0;
        dup[23] = 0;   // leaf 7 = leaf 0
        ok(!check_octree(1, 8, dup.data()).empty(), "duplicate refused");
        std::vector<uint16_t> out = {0, 2, 0, 0, 0, 0};   // x = 2 outside 2^1
        ok(!check_octree(1, 2, out.data()).empty(), "cell outside the grid refused");
        std::vector<uint16_t> big = {511, 0, 511, 0, 511, 0};
        ok(check_octree(9, 2, big.data()).empty(), "depth-9 corner cells accepted");
    }
    // ---- skin ---------------------------------------------------------------------
    {
        const int64_t n = 3;
        std::vector<uint8_t> bone = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12};   // [4][n]
        std::vector<float> w = {0.1f, 0.5f, 0.25f, 0.6f, 0.5f, 0.25f, 0.2f, 0.0f, 0.25f, 0.1f, 0.0f, 0.25f};
        int mb = -1;
        std::vector<uint8_t> dom;
        ok(check_skin(n, bone.data(), w.data(), &mb, &dom).empty(), "skin accepted");
        ok(mb == 12, "largest bone id");
        // leaf 0: weights 0.1, 0.6, 0.2, 0.1 -> slot 1 (bone 4); leaf 1: 0.5, 0.5
        // -> the first (bone 2); leaf 2: all equal -> the first (bone 3)
        ok(dom.size() == 3 && dom[0] == 4 && dom[1] == 2 && dom[2] == 3, "dominant bones");
        std::vector<float> bad = w;
        bad[4] = -1e-6f;
        ok(!check_skin(n, bone.data(), bad.data(), &mb, &dom).empty(), "negative weight refused");
        bad[4] = std::numeric_limits<float>::quiet_NaN();
        ok(!check_skin(n, bone.data(), bad.data(), &mb, &dom).empty(), "NaN weight refused");
        bad[4] = std::numeric_limits<float>::infinity();
        ok(!check_skin(n, bone.data(), bad.data(), &mb, &dom).empty(), "infinite weight refused");
        ok(!check_skin(n, nullptr, w.data(), &mb, &dom).empty(), "NULL bones refused");
    }
    // ---- skeleton -----------------------------------------------------------------
    {
        std::vector<int32_t> par = {-1, 0, 1, 1, 0};
        std::vector<double> rest(15, 0.25);
        ok(check_skeleton(5, par.data(), rest.data()).empty(), "tree accepted");
        std::vector<int32_t> p255(255);
        std::vector<double> r255(765, 0.0);
        p255[0] = -1;
        for (int j = 1; j < 255; ++j) p255[j] = j - 1;   // a 255-deep chain
        ok(check_skeleton(255, p255.data(), r255.data()).empty(), "255 joints accepted");
        ok(!check_skeleton(256, p255.data(), r255.data()).empty(), "256 joints refused");
        ok(!check_skeleton(0, par.data(), rest.data()).empty(), "no joints refused");
        std::vector<int32_t> bp = par;
        bp[0] = 0;
        ok(!check_skeleton(5, bp.data(), rest.data()).empty(), "root with a parent refused");
        bp = par;
        bp[3] = 3;
        ok(!check_skeleton(5, bp.data(), rest.data()).empty(), "parent not before the child refused");
        std::vector<double> br = rest;
        br[7] = nan;
        ok(!check_skeleton(5, par.data(), br.data()).empty(), "NaN joint refused");
    }
    // ---- poses --------------------------------------------------------------------
    {
        const int J = 2, P = 2;
        std::vector<double> r(P * J * 3), R(P * 3), T(P * 3), buf;
        for (size_t i = 0; i < r.size(); ++i) r[i] = 0.01 * (double)i;
        for (int i = 0; i < P * 3; ++i) {
            R[i] = 1.0 + i;
            T[i] = 10.0 + i;
        }
        ok(pack_poses(J, P, r.data(), R.data(), T.data(), &buf).empty(), "poses accepted");
        ok(buf.size() == (size_t)P * (J + 2) * 3, "packed size");
        // pose 1: r_0, r_1, R, T
        ok(buf[12] == r[6] && buf[17] == r[11] && buf[18] == R[3] && buf[23] == T[5], "packed layout");
        ok(!pack_poses(J, 0, r.data(), R.data(), T.data(), &buf).empty(), "P = 0 refused");
        ok(!pack_poses(J, 4097, r.data(), R.data(), T.data(), &buf).empty(), "P = 4097 refused");
        T[4] = std::numeric_limits<double>::infinity();
        ok(!pack_poses(J, P, r.data(), R.data(), T.data(), &buf).empty(), "infinite translation refused");
    }
    // ---- cameras ------------------------------------------------------------------
    {
        const double K[9] = {100, 0, 32, 0, 120, 24, 0, 0, 1};
        const double c = std::cos(0.3), s = std::sin(0.3);
        const double M[12] = {c, -s, 0, 0.5, s, c, 0, -0.25, 0, 0, 1, 3.0};
        std::vector<CamParams> cams;
        ok(check_cameras(1, 48, 64, K, M, &cams).empty(), "camera accepted");
        ok(cams.size() == 1 && cams[0].fx == 100 && cams[0].fy == 120 && cams[0].cx == 32 && cams[0].cy == 24,
           "intrinsics");
        ok(cams[0].R[1] == -s && cams[0].R[3] == s && cams[0].t[2] == 3.0, "rotation and centre");
        ok(check_cameras(1, 8192, 1, K, M, &cams).empty(), "8192 x 1 accepted");
        ok(!check_cameras(1, 8193, 64, K, M, &cams).empty(), "H = 8193 refused");
        ok(!check_cameras(0, 48, 64, K, M, &cams).empty(), "V = 0 refused");
        double M2[12];
        for (int i = 0; i < 12; ++i) M2[i] = M[i];
        M2[0] *= 1.001;   // not orthonormal
        ok(!check_cameras(1, 48, 64, K, M2, &cams).empty(), "scaled rotation refused");
        double K2[9];
        for (int i = 0; i < 9; ++i) K2[i] = K[i];
        K2[4] = 0.0;
        ok(!check_cameras(1, 48, 64, K2, M, &cams).empty(), "zero focal length refused");
        K2[4] = nan;
        ok(!check_cameras(1, 48, 64, K2, M, &cams).empty(), "NaN focal length refused");
        ok(!check_cameras(1, 48, 64, nullptr, M, &cams).empty(), "NULL K refused");
    }
    if (fails) return 1;
    std::printf("validate sanitizer driver: all checks passed\n");
    return 0;
}
