/*
 * Host sanitizer driver of the FP64 oracle (ray_oracle.c): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py
 * and run on a small posed grid.  Every entry point is called with all of its
 * optional outputs; the results are checked against facts that hold for any
 * input (A + T_final = 1 without the early stop, hit counts within the list
 * capacity) and the closed form of an axis-aligned column (Eq. 5-6 with
 * chords of one leaf edge: A = 1 - exp(-h sum sigma)).  Exit status 0 when
 * every check passes.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_render(int64_t n, const double* o, const double* d, int G, double h, int64_t M, const int64_t* occ_key,
                  const int64_t* occ_leaf, int C, const double* sigma, const double* feat, double lambda_th,
                  double* F, double* A, double* Tfin, int32_t* n_comp, int32_t* n_hit, double* min_gap,
                  double* min_tgap, int max_hits, int64_t* hit_leaf, double* hit_delta, double* seg,
                  double depth_sigma, double* depth, int n_threads);
int oracle_render_sh(int64_t n, const double* o, const double* d, int G, double h, int64_t M,
                     const int64_t* occ_key, const int64_t* occ_leaf, int C, int H, const double* sigma,
                     const double* feat, const int32_t* dom_bone, const double* rot, double lambda_th, double* F,
                     double* A, double* Tfin, double* min_gap, double* min_tgap, int n_threads);
int oracle_backward(int64_t n, const double* o, const double* d, int G, double h, int64_t M,
                    const int64_t* occ_key, const int64_t* occ_leaf, int C, const double* sigma,
                    const double* feat, double lambda_th, const double* gF, const double* gA, double* dsigma,
                    double* dfeat, int n_threads);
void oracle_sh_basis(int H, double x, double y, double z, double* Y);

enum { G = 8, C = 4, NRAY = 9, MAXH = 3, SH = 9 };

static uint64_t lcg = 12345u;
static double urand(void) {   /* uniform in [0, 1) */
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
static void check(int ok, const char* what) {
    if (!ok) {
        fprintf(stderr, "check failed: %s\n", what);
        ++fails;
    }
}

int main(void) {
    const double h = 2.0 / G;
    /* occupied posed cells (linear keys (z G + y) G + x, ascending): a column
     * x = 2..5 at y = 3, z = 4, and three scattered cells */
    int64_t key[16], leaf[16];
    int64_t M = 0;
    for (int x = 2; x <= 5; ++x) key[M++] = (4 * G + 3) * G + x;
    key[M++] = (1 * G + 1) * G + 1;
    key[M++] = (6 * G + 5) * G + 2;
    key[M++] = (7 * G + 7) * G + 7;
    for (int i = 0; i < M; ++i)   /* sort ascending */
        for (int j = i + 1; j < M; ++j)
            if (key[j] < key[i]) {
                int64_t t = key[i];
                key[i] = key[j];
                key[j] = t;
            }
    const int N = (int)M + 2;   /* two leaves lost their cells to collisions */
    for (int i = 0; i < M; ++i) leaf[i] = i;
    double sigma[16], feat[16 * C], featsh[16 * SH * C];
    int32_t dom[16];
    for (int i = 0; i < N; ++i) {
        sigma[i] = 0.5 + 4.0 * urand();
        for (int c = 0; c < C; ++c) feat[i * C + c] = 2.0 * urand() - 1.0;
        for (int k = 0; k < SH * C; ++k) featsh[i * SH * C + k] = 2.0 * urand() - 1.0;
        dom[i] = i % 2;
    }
    double rot[2 * 9] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, -1, 0, 1, 0, 0, 0, 0, 1};
    /* rays: along +x through the column (cell centres), oblique ones, a miss,
     * one starting inside the root, axis-parallel ones with zero components */
    double o[NRAY * 3], d[NRAY * 3];
    const double yc = -1.0 + 3.5 * h, zc = -1.0 + 4.5 * h;
    double rays[NRAY][6] = {
        {-3.0, yc, zc, 1.0, 0.0, 0.0},
        {-2.0, -1.7, -1.9, 0.6, 0.5, 0.62},
        {2.5, 2.1, -0.3, -0.7, -0.55, 0.1},
        {0.0, 5.0, 0.0, 0.0, 0.0, 1.0},            /* misses the root */
        {0.05, 0.07, -0.02, 0.3, -0.8, 0.5},       /* inside the root */
        {-1.0 + 1.5 * h, -1.0 + 1.5 * h, -4.0, 0.0, 0.0, 1.0},
        {-1.0 + 2.5 * h, -3.0, -1.0 + 6.5 * h, 0.0, 1.0, 0.0},
        {1.9, 1.8, 1.7, -0.57, -0.58, -0.58},
        {-1.5, -1.2, 0.1, 0.8, 0.55, 0.05},
    };
    for (int r = 0; r < NRAY; ++r) {
        double nn = 0.0;
        for (int a = 0; a < 3; ++a) nn += rays[r][3 + a] * rays[r][3 + a];
        nn = sqrt(nn);
        for (int a = 0; a < 3; ++a) {
            o[3 * r + a] = rays[r][a];
            d[3 * r + a] = rays[r][3 + a] / nn;
        }
    }
    double F[NRAY * C], A[NRAY], T[NRAY], gap[NRAY], tgap[NRAY], seg[NRAY * 4], dep[NRAY];
    int32_t ncomp[NRAY], nhit[NRAY];
    int64_t hl[NRAY * MAXH];
    double hd[NRAY * MAXH];
    for (int pass = 0; pass < 2; ++pass) {
        const double lam = pass ? 0.3 : 0.0;
        check(oracle_render(NRAY, o, d, G, h, M, key, leaf, C, sigma, feat, lam, F, A, T, ncomp, nhit, gap, tgap,
                            MAXH, hl, hd, seg, 1.5, dep, 1) == 0,
              "oracle_render status");
        for (int r = 0; r < NRAY; ++r) {
            check(ncomp[r] <= nhit[r], "composited <= hit");
            if (pass == 0) check(fabs(A[r] + T[r] - 1.0) < 1e-12, "A + T = 1 without the early stop");
            if (pass == 1 && ncomp[r] < nhit[r]) check(T[r] < lam, "early stop below lambda");
        }
    }
    /* the column ray: four chords of one leaf edge */
    {
        double tau = 0.0;
        for (int m = 0; m < M; ++m)
            if (key[m] / (G * G) == 4 && (key[m] / G) % G == 3) tau += sigma[leaf[m]] * h;
        oracle_render(1, o, d, G, h, M, key, leaf, C, sigma, feat, 0.0, F, A, T, ncomp, nhit, gap, tgap, 0, NULL,
                      NULL, NULL, INFINITY, NULL, 1);
        check(ncomp[0] == 4, "column: four samples");
        check(fabs(A[0] - (1.0 - exp(-tau))) < 1e-12, "column: closed-form opacity");
    }
    check(oracle_render(0, o, d, G, h, M, key, leaf, C, sigma, feat, 0.01, F, A, T, ncomp, nhit, gap, tgap, 0, NULL,
                        NULL, NULL, 0.0, NULL, 1) == 0,
          "empty ray set");
    double Fs[NRAY * C], As[NRAY], Ts[NRAY];
    check(oracle_render_sh(NRAY, o, d, G, h, M, key, leaf, C, SH, sigma, featsh, dom, rot, 0.01, Fs, As, Ts, gap,
                           tgap, 1) == 0,
          "oracle_render_sh status");
    double Y[9];
    oracle_sh_basis(SH, 0.0, 0.0, 1.0, Y);
    check(fabs(Y[0] - 0.28209479177387814) < 1e-15, "Y_00");
    double gF[NRAY * C], gA[NRAY], ds[16] = {0}, df[16 * C] = {0};
    for (int i = 0; i < NRAY * C; ++i) gF[i] = urand() - 0.5;
    for (int i = 0; i < NRAY; ++i) gA[i] = urand() - 0.5;
    check(oracle_backward(NRAY, o, d, G, h, M, key, leaf, C, sigma, feat, 0.01, gF, gA, ds, df, 1) == 0,
          "oracle_backward status");
    check(oracle_backward(NRAY, o, d, G, h, M, key, leaf, C, sigma, feat, 0.0, gF, NULL, ds, df, 1) == 0,
          "oracle_backward without dL/dA");
    for (int i = M; i < N; ++i) check(ds[i] == 0.0, "losers get no gradient");
    if (fails) return 1;
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
