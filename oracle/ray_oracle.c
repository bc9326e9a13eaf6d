/*
 * FP64 CPU oracle for ray indexing and compositing over a posed voxel set.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * definition that the GPU renderer is checked against.  It shares no code with
 * the GPU path and must never be linked into, or called by, the product
 * library.
 *
 * What it computes, per ray (Section 3.1 "Dynamic Volume Rendering",
 * Eq. 5 and Eq. 6, with the readings listed below):
 *
 *  1. Clip the ray o + t d (|d| = 1) to the posed root box [-1,1]^3:
 *     t_a = max(t_entry, 0), t_b = t_exit.  A miss gives F = 0, A = 0, T = 1.
 *  2. Partition (t_a, t_b) by every lattice-plane crossing
 *     t = (-1 + k h - o_a) / d_a on each axis a with d_a != 0 (qsort, equal
 *     values merged).  Each positive-length segment (s, s') lies in the cell
 *     floor((o + (s+s')/2 d + 1) / h) (midpoint rule).  If that cell is
 *     occupied, the segment is one sample: the winner leaf of the cell and
 *     delta = s' - s, the length of the ray inside the voxel.
 *  3. Composite front to back with the *exclusive* transmittance
 *     T_i = exp(-sum_{j<i} sigma_j delta_j):
 *        alpha_i = 1 - exp(-sigma_i delta_i),  w_i = T_i alpha_i,
 *        F += w_i f_i,  A += w_i,  T_{i+1} = T_i exp(-sigma_i delta_i),
 *     and stop right after the sample at which T < lambda_th (the early stop
 *     of Section 3.1 at accumulated alpha > 1 - lambda_th; the crossing sample
 *     is included).
 *
 * The adjoint (oracle_backward) differentiates L with respect to the leaf
 * densities and features through step 3, holding the set of composited samples
 * fixed, with explicit suffix sums computed by a reverse pass:
 *   dL/df_i     = w_i g
 *   dL/dsigma_i = delta_i [ g . (T_{i+1} f_i - S_i) + g_A T_final ],
 *   S_i = sum_{k>i} w_k f_k,   g = dL/dF,  g_A = dL/dA.
 *
 * Cells are identified by the linear key (cz*G + cy)*G + cx; the occupied set
 * is passed as sorted keys with their winner leaf ids, and looked up by
 * binary search.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* binary search in a sorted key array; returns index or -1 */
static int64_t find_key(const int64_t* keys, int64_t n, int64_t key) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == key) return mid;
        if (keys[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Clip to [-1,1]^3.  Returns 1 and sets [*ta, *tb] with *tb > *ta on a hit. */
static int clip_root(const double o[3], const double d[3], double* ta, double* tb) {
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < -1.0 || o[a] > 1.0) return 0;
            continue;
        }
        double u = (-1.0 - o[a]) / d[a];
        double v = (1.0 - o[a]) / d[a];
        if (u > v) { double s = u; u = v; v = s; }
        if (u > t0) t0 = u;
        if (v < t1) t1 = v;
    }
    if (t0 < 0.0) t0 = 0.0;
    if (!(t1 > t0)) return 0;
    *ta = t0;
    *tb = t1;
    return 1;
}

typedef struct {
    int64_t leaf;   /* winner leaf id */
    double delta;   /* chord length */
    double t0, t1;  /* the segment (t0, t1) of the ray inside the voxel */
} sample_t;

/* Enumerate the occupied samples of one ray in increasing t.
 * Writes up to cap samples into out; returns the total number found.
 * *min_gap receives the smallest gap between consecutive partition points
 * (0 if two crossings coincided exactly), a guard band for rounding. */
static int64_t ray_samples(const double o[3], const double d[3], int G, double h,
                           int64_t M, const int64_t* occ_key, const int64_t* occ_leaf,
                           sample_t* out, int64_t cap, double* pts, double* min_gap,
                           double* ta_out, double* tb_out) {
    double ta, tb;
    *min_gap = INFINITY;
    *ta_out = NAN;
    *tb_out = NAN;
    if (!clip_root(o, d, &ta, &tb)) return 0;
    *ta_out = ta;
    *tb_out = tb;
    int64_t np = 0;
    pts[np++] = ta;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        for (int k = 0; k <= G; ++k) {
            double t = (-1.0 + k * h - o[a]) / d[a];
            if (t > ta && t < tb) pts[np++] = t;
        }
    }
    pts[np++] = tb;
    qsort(pts, (size_t)np, sizeof(double), cmp_double);
    int64_t ns = 0;
    for (int64_t i = 0; i + 1 < np; ++i) {
        double s0 = pts[i], s1 = pts[i + 1];
        double gap = s1 - s0;
        if (gap < *min_gap) *min_gap = gap;
        if (!(s1 > s0)) continue;          /* equal crossings merge */
        double mid = 0.5 * (s0 + s1);
        int64_t c[3];
        int inside = 1;
        for (int a = 0; a < 3; ++a) {
            c[a] = (int64_t)floor((o[a] + mid * d[a] + 1.0) / h);
            if (c[a] < 0 || c[a] >= G) inside = 0;
        }
        if (!inside) continue;
        int64_t key = (c[2] * G + c[1]) * (int64_t)G + c[0];
        int64_t idx = find_key(occ_key, M, key);
        if (idx < 0) continue;
        if (ns < cap) {
            out[ns].leaf = occ_leaf[idx];
            out[ns].delta = s1 - s0;
            out[ns].t0 = s0;
            out[ns].t1 = s1;
        }
        ++ns;
    }
    return ns;
}

static int64_t max_points(int G) { return 3 * (int64_t)(G + 1) + 2; }

/*
 * Forward render of n rays.  Outputs (all per ray, caller-allocated):
 *   F [n][C], A [n], Tfin [n], n_comp [n] (composited samples), n_hit [n]
 *   (all occupied samples, ignoring the early stop), min_gap [n] (rounding
 *   guard band of the partition), min_tgap [n] (smallest |T - lambda| / lambda
 *   over the composited samples; +inf when lambda == 0).
 * Optional hit lists (hit_leaf/hit_delta [n][max_hits], may be NULL) record the
 * composited samples in order.  Optional seg [n][4] (may be NULL) receives
 * t_a, t_b of the clipped ray (NaN on a miss), the entry t of the first
 * composited sample and the exit t of the last one (NaN without samples): the
 * interval a ray-interval proposal has to cover.
 * Optional depth [n] (may be NULL) receives the depth-buffer value of the
 * hybrid rendering (Section 3.1, paragraph "Hybrid Rendering"): the ray is
 * traced through the whole clipped span, and the value is the distance t
 * along the unit ray at which it enters the first occupied voxel (the
 * collision winner of its cell) whose density is above depth_sigma; +inf
 * when there is none.  The early stop of the compositing does not end this
 * search.
 * Returns 0, or -1 on allocation failure.
 */
int oracle_render(int64_t n, const double* o, const double* d, int G, double h,
                  int64_t M, const int64_t* occ_key, const int64_t* occ_leaf,
                  int C, const double* sigma, const double* feat, double lambda_th,
                  double* F, double* A, double* Tfin, int32_t* n_comp, int32_t* n_hit,
                  double* min_gap, double* min_tgap,
                  int max_hits, int64_t* hit_leaf, double* hit_delta, double* seg,
                  double depth_sigma, double* depth, int n_threads) {
    int failed = 0;
    int64_t cap = max_points(G);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        double* pts = (double*)malloc(sizeof(double) * (size_t)cap);
        sample_t* smp = (sample_t*)malloc(sizeof(sample_t) * (size_t)cap);
        if (!pts || !smp) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t r = 0; r < n; ++r) {
                double gap, ta, tb;
                int64_t ns = ray_samples(o + 3 * r, d + 3 * r, G, h, M, occ_key, occ_leaf,
                                         smp, cap, pts, &gap, &ta, &tb);
                double T = 1.0, acc = 0.0, tg = INFINITY, dep = INFINITY;
                double* Fr = F + (size_t)r * C;
                for (int c = 0; c < C; ++c) Fr[c] = 0.0;
                /* depth buffer: first occupied voxel of the whole ray above the threshold */
                for (int64_t i = 0; i < ns; ++i) {
                    if (sigma[smp[i].leaf] > depth_sigma) {
                        dep = smp[i].t0;
                        break;
                    }
                }
                int64_t used = 0;
                for (int64_t i = 0; i < ns; ++i) {
                    const double s = sigma[smp[i].leaf];
                    const double* f = feat + (size_t)smp[i].leaf * C;
                    double tau = s * smp[i].delta;
                    double alpha = -expm1(-tau);
                    double w = T * alpha;
                    for (int c = 0; c < C; ++c) Fr[c] += w * f[c];
                    acc += w;
                    T = T * exp(-tau);
                    if (hit_leaf && used < max_hits) {
                        hit_leaf[(size_t)r * max_hits + used] = smp[i].leaf;
                        hit_delta[(size_t)r * max_hits + used] = smp[i].delta;
                    }
                    ++used;
                    if (lambda_th > 0.0) {
                        double g = fabs(T - lambda_th) / lambda_th;
                        if (g < tg) tg = g;
                    }
                    if (T < lambda_th) break;
                }
                A[r] = acc;
                Tfin[r] = T;
                if (depth) depth[r] = dep;
                if (seg) {
                    double* sg = seg + 4 * (size_t)r;
                    sg[0] = ta;
                    sg[1] = tb;
                    sg[2] = used > 0 ? smp[0].t0 : NAN;
                    sg[3] = used > 0 ? smp[used - 1].t1 : NAN;
                }
                n_comp[r] = (int32_t)used;
                n_hit[r] = (int32_t)ns;
                min_gap[r] = gap;
                min_tgap[r] = tg;
            }
        }
        free(pts);
        free(smp);
    }
    return failed ? -1 : 0;
}

/*
 * Real spherical-harmonic basis Y_0 .. Y_{H-1} (H = 1, 4 or 9: degrees 0, 1,
 * 2) at the unit direction (x, y, z): the orthonormal real harmonics,
 * ordered by degree l and then m = -l .. l, without the Condon-Shortley
 * phase:  l = 0: 1/(2 sqrt(pi));  l = 1: sqrt(3/(4 pi)) * (y, z, x);
 * l = 2: sqrt(15/pi)/2 * xy, sqrt(15/pi)/2 * yz, sqrt(5/pi)/4 * (3z^2 - 1),
 *        sqrt(15/pi)/2 * xz, sqrt(15/pi)/4 * (x^2 - y^2).
 */
void oracle_sh_basis(int H, double x, double y, double z, double* Y) {
    const double pi = 3.14159265358979323846;
    Y[0] = 0.5 / sqrt(pi);
    if (H < 4) return;
    const double c1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = c1 * y;
    Y[2] = c1 * z;
    Y[3] = c1 * x;
    if (H < 9) return;
    const double c2 = 0.5 * sqrt(15.0 / pi);
    Y[4] = c2 * x * y;
    Y[5] = c2 * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    Y[7] = c2 * x * z;
    Y[8] = 0.5 * c2 * (x * x - y * y);
}

/*
 * Eq. 5 with view-dependent features (Eq. 2): as oracle_render (without the
 * debug outputs), but sample i contributes w_i S(f_i, d^c) with
 * S_c = sum_h k_{h,c} Y_h(d^c), the coefficients feat [N][H][C] of the
 * winner leaf, and the canonical direction d^c = R^T d of the ray's unit
 * direction d, R the rotation (row-major 3x3, rot [J][9]) of the leaf's
 * dominant bone dom_bone [N] (the reading of the voxel rotation R_i^t).
 */
int oracle_render_sh(int64_t n, const double* o, const double* d, int G, double h,
                     int64_t M, const int64_t* occ_key, const int64_t* occ_leaf,
                     int C, int H, const double* sigma, const double* feat, const int32_t* dom_bone,
                     const double* rot, double lambda_th, double* F, double* A, double* Tfin,
                     double* min_gap, double* min_tgap, int n_threads) {
    int failed = 0;
    int64_t cap = max_points(G);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        double* pts = (double*)malloc(sizeof(double) * (size_t)cap);
        sample_t* smp = (sample_t*)malloc(sizeof(sample_t) * (size_t)cap);
        if (!pts || !smp) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t r = 0; r < n; ++r) {
                double gap, ta, tb;
                const double* dr = d + 3 * r;
                int64_t ns = ray_samples(o + 3 * r, dr, G, h, M, occ_key, occ_leaf, smp, cap, pts, &gap, &ta, &tb);
                double T = 1.0, acc = 0.0, tg = INFINITY;
                double* Fr = F + (size_t)r * C;
                for (int c = 0; c < C; ++c) Fr[c] = 0.0;
                for (int64_t i = 0; i < ns; ++i) {
                    const int64_t leaf = smp[i].leaf;
                    const double* R = rot + 9 * (size_t)dom_bone[leaf];
                    double dc[3], Y[9];
                    for (int a = 0; a < 3; ++a) dc[a] = R[a] * dr[0] + R[3 + a] * dr[1] + R[6 + a] * dr[2];
                    oracle_sh_basis(H, dc[0], dc[1], dc[2], Y);
                    const double s = sigma[leaf];
                    const double tau = s * smp[i].delta;
                    const double w = T * -expm1(-tau);
                    for (int c = 0; c < C; ++c) {
                        double S = 0.0;
                        for (int k = 0; k < H; ++k) S += feat[((size_t)leaf * H + k) * C + c] * Y[k];
                        Fr[c] += w * S;
                    }
                    acc += w;
                    T = T * exp(-tau);
                    if (lambda_th > 0.0) {
                        double g = fabs(T - lambda_th) / lambda_th;
                        if (g < tg) tg = g;
                    }
                    if (T < lambda_th) break;
                }
                A[r] = acc;
                Tfin[r] = T;
                min_gap[r] = gap;
                min_tgap[r] = tg;
            }
        }
        free(pts);
        free(smp);
    }
    return failed ? -1 : 0;
}

/*
 * Adjoint of oracle_render for the loss whose gradients with respect to the
 * outputs are gF [n][C] and gA [n] (gA may be NULL for zero).  Accumulates
 * (+=) into dsigma [N] and dfeat [N][C].  Returns 0 or -1.
 */
int oracle_backward(int64_t n, const double* o, const double* d, int G, double h,
                    int64_t M, const int64_t* occ_key, const int64_t* occ_leaf,
                    int C, const double* sigma, const double* feat, double lambda_th,
                    const double* gF, const double* gA, double* dsigma, double* dfeat,
                    int n_threads) {
    int failed = 0;
    int64_t cap = max_points(G);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        double* pts = (double*)malloc(sizeof(double) * (size_t)cap);
        sample_t* smp = (sample_t*)malloc(sizeof(sample_t) * (size_t)cap);
        double* w = (double*)malloc(sizeof(double) * (size_t)cap);
        double* Tn = (double*)malloc(sizeof(double) * (size_t)cap);
        double* S = (double*)malloc(sizeof(double) * (size_t)C);
        if (!pts || !smp || !w || !Tn || !S) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t r = 0; r < n; ++r) {
                double gap, ta, tb;
                int64_t ns = ray_samples(o + 3 * r, d + 3 * r, G, h, M, occ_key, occ_leaf,
                                         smp, cap, pts, &gap, &ta, &tb);
                /* forward: weights and transmittances of the composited samples */
                double T = 1.0;
                int64_t used = 0;
                for (int64_t i = 0; i < ns; ++i) {
                    double tau = sigma[smp[i].leaf] * smp[i].delta;
                    w[i] = T * (-expm1(-tau));
                    T = T * exp(-tau);
                    Tn[i] = T;
                    ++used;
                    if (T < lambda_th) break;
                }
                const double Tfinal = T;
                const double* g = gF + (size_t)r * C;
                const double ga = gA ? gA[r] : 0.0;
                /* reverse pass with the explicit suffix sum S_i = sum_{k>i} w_k f_k */
                for (int c = 0; c < C; ++c) S[c] = 0.0;
                for (int64_t i = used - 1; i >= 0; --i) {
                    const int64_t leaf = smp[i].leaf;
                    const double* f = feat + (size_t)leaf * C;
                    double ds = 0.0;
                    for (int c = 0; c < C; ++c) ds += g[c] * (Tn[i] * f[c] - S[c]);
                    ds = smp[i].delta * (ds + ga * Tfinal);
#ifdef _OPENMP
#pragma omp atomic
#endif
                    dsigma[leaf] += ds;
                    for (int c = 0; c < C; ++c) {
                        double v = w[i] * g[c];
#ifdef _OPENMP
#pragma omp atomic
#endif
                        dfeat[(size_t)leaf * C + c] += v;
                    }
                    for (int c = 0; c < C; ++c) S[c] += w[i] * f[c];
                }
            }
        }
        free(pts);
        free(smp);
        free(w);
        free(Tn);
        free(S);
    }
    return failed ? -1 : 0;
}

/* Number of OpenMP threads the oracle would use by default. */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
