/*
 * CPU oracle for LOD Gaussian-splatting per-frame rendering.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Plain, slow, obviously correct: one Gaussian / one pixel at a time, in the
 * order the paper states the method.  The same source is compiled twice:
 *   -DREAL=float   (liblodge_oracle_f32.so): decisions (selection, tile
 *                  rectangles, sort keys, compositing thresholds) in FP32,
 *                  the precision the renderer works in;
 *   -DREAL=double  (liblodge_oracle_f64.so): the same definition in FP64,
 *                  used for the adjoint and finite differences.
 * Build with -O2 -ffp-contract=off (no FMA contraction, no fast-math) so
 * every +,-,*,/,sqrt is one IEEE-rounded operation, evaluated left to right
 * exactly as written.
 *
 * Passages followed (LODGE, arXiv 2505.23158):
 *   Sec. 3 "Preliminaries: 3D Gaussian Splatting", Eq. 1  -- splatting, alpha,
 *          16x16 tiles, per-tile depth sort, front-to-back blending
 *   Sec. 3 "Level of Detail (LOD) representation", Eq. 2  -- active set
 *   Sec. 3 "Building LOD representation", Eq. 3          -- 3-D smoothing filter
 *   Sec. 3 "Reducing memory with chunk-based rendering"   -- per-chunk active
 *          sets with thresholds offset by the chunk radius
 *   Sec. 3 "Opacity blending ...", Eq. 4                  -- two nearest chunks,
 *          projection weight t, opacity modulation of the symmetric difference
 *   Supp. "Details on training the full representation"   -- 2-D filter of the
 *          renderer (Mip-Splatting style)
 * Where the paper is silent or garbled, the reading taken is stated at each
 * use below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL float
#endif
typedef REAL real;

#define IS_F32 (sizeof(real) == 4)
#define R_SQRT(x) (IS_F32 ? (real)sqrtf((float)(x)) : (real)sqrt((double)(x)))
#define R_EXP(x) (IS_F32 ? (real)expf((float)(x)) : (real)exp((double)(x)))
#define R_FLOOR(x) (IS_F32 ? (real)floorf((float)(x)) : (real)floor((double)(x)))
#define R_CEIL(x) (IS_F32 ? (real)ceilf((float)(x)) : (real)ceil((double)(x)))

#define TILE 16
#define NSH 16

/* The timing build of the benchmark's CPU baseline compiles this same source
 * with -fopenmp: ORC_PARALLEL_FOR then spreads the independent per-Gaussian
 * projections and per-pixel walks over the host cores.  Each iteration writes
 * only its own outputs, so the results are those of the plain builds; the
 * arithmetic is untouched.  Without -fopenmp it expands to nothing. */
#ifdef _OPENMP
#define ORC_PARALLEL_FOR _Pragma("omp parallel for schedule(dynamic, 256)")
#define ORC_PARALLEL_ROWS _Pragma("omp parallel for schedule(dynamic, 1)")
#else
#define ORC_PARALLEL_FOR
#define ORC_PARALLEL_ROWS
#endif

/* ------------------------------------------------------------------------ */
/* inputs                                                                   */
/* ------------------------------------------------------------------------ */

/* One LOD level G^(l): structure of arrays, activated parameters.
 * mean[3][n], scale[3][n] (linear), quat[4][n] (w,x,y,z, used as given),
 * opacity[n], sh[16][3][n]; filter3d_var is the Eq. 3 filter variance. */
typedef struct {
    int64_t n;
    const real *mean, *scale, *quat, *opacity, *sh;
    int32_t sh_degree;
    real filter3d_var;
} orc_level;

/* Pinhole camera, OpenCV axes: R is world->camera (row-major), t its
 * translation, pos the camera centre (given explicitly). */
typedef struct {
    int32_t width, height;
    real fx, fy, cx, cy;
    real R[9], t[3], pos[3];
    real znear, lim_x, lim_y;
    real bg[3];
} orc_camera;

/* gradient planes for one level, same shapes as the parameters (+=) */
typedef struct {
    real *mean, *scale, *quat, *opacity, *sh;
} orc_grads;

enum { ORC_ALL = 0, ORC_LOD_CAMERA = 1, ORC_CHUNKED = 2 };

static real sq(real x) { return x * x; }

static real dist2(const real* p, const real* q)
{
    /* ((px-qx)^2 + (py-qy)^2) + (pz-qz)^2, left to right */
    real dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* ------------------------------------------------------------------------ */
/* Eq. 4: the two nearest chunk centres and the projection weight t          */
/* ------------------------------------------------------------------------ */

/* f = nearest centre, o = second nearest (lowest index wins ties; the paper
 * does not say).  t_bar = ((c - m_o) . (m_f - m_o)) / |m_o - m_f|^2, the
 * normalised length of the projection of c - m_o onto the centre line.
 * Reading of the configs' "blend bands": with band > 0 the ramp is narrowed
 * to a strip of that width around the bisector, t_bar <- 0.5 + (t_bar - 0.5)
 * * |m_f - m_o| / band; band <= 0 (or band = |m_f - m_o|) is Eq. 4 as printed.
 * t = min(1, max(0, t_bar)).  K = 1: f = 0, o = -1, t = 1. */
int orc_chunk_pair(const real* centers, int32_t K, real band, const real* c,
                   int32_t* f_out, int32_t* o_out, real* t_out)
{
    if (K < 1) return -1;
    int32_t f = 0;
    real df = dist2(c, centers);
    for (int32_t k = 1; k < K; k++) {
        real dk = dist2(c, centers + 3 * k);
        if (dk < df) { df = dk; f = k; }
    }
    if (K == 1) { *f_out = f; *o_out = -1; *t_out = (real)1; return 0; }
    int32_t o = -1;
    real dbest = 0;
    for (int32_t k = 0; k < K; k++) {
        if (k == f) continue;
        real dk = dist2(c, centers + 3 * k);
        if (o < 0 || dk < dbest) { dbest = dk; o = k; }
    }
    const real* mf = centers + 3 * f;
    const real* mo = centers + 3 * o;
    real g[3] = {mf[0] - mo[0], mf[1] - mo[1], mf[2] - mo[2]};
    real e[3] = {c[0] - mo[0], c[1] - mo[1], c[2] - mo[2]};
    real num = (e[0] * g[0] + e[1] * g[1]) + e[2] * g[2];
    real den = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
    real tb = num / den;
    if (band > 0) tb = (real)0.5 + (tb - (real)0.5) * (R_SQRT(den) / band);
    real t = tb;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    *f_out = f; *o_out = o; *t_out = t;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 2 (+ chunk offsets): active set selection                             */
/* ------------------------------------------------------------------------ */

/* Squared distance bounds of level l about a centre whose thresholds are
 * offset by r (r = 0 about the camera):  lo(0) = 0, lo(l) = (d_l + r)^2,
 * hi(l) = lo(l+1), hi(L-1) = +inf.  Interval [lo, hi): inclusive lower,
 * exclusive upper, as Eq. 2 prints it. */
static void bounds(const real* d, int32_t L, int32_t l, real r, real* lo, real* hi)
{
    *lo = (l == 0) ? (real)0 : sq(d[l - 1] + r);
    *hi = (l == L - 1) ? (real)INFINITY : sq(d[l] + r);
}

/* Selects, in ascending global id (id = sum_{j<l} n_j + i), every Gaussian
 * of the active set and its opacity weight:
 *   ALL:        every Gaussian of every level, w = 1;
 *   LOD_CAMERA: Eq. 2 about the camera centre, w = 1;
 *   CHUNKED:    Eq. 2 about each of the two nearest chunk centres with the
 *               distances offset by that chunk's r_k; the union is emitted
 *               with w = 1 in both sets, t in A_f only, 1 - t in A_o only
 *               (Eq. 4: only the symmetric difference is re-weighted).
 * Writes min(count, cap) entries and returns count (-1 on bad arguments). */
int64_t orc_select(const orc_level* lv, int32_t L, const real* d, int32_t mode,
                   const real* centers, const real* offsets, int32_t K, real band,
                   const real* pos, uint32_t* ids, real* w, int64_t cap,
                   int32_t* f_out, int32_t* o_out, real* t_out)
{
    int32_t f = -1, o = -1;
    real t = 1;
    if (mode == ORC_CHUNKED) {
        if (orc_chunk_pair(centers, K, band, pos, &f, &o, &t) != 0) return -1;
    }
    if (f_out) *f_out = f;
    if (o_out) *o_out = o;
    if (t_out) *t_out = t;
    real t_o = (real)1 - t;
    int64_t count = 0, base = 0;
    for (int32_t l = 0; l < L; l++) {
        real lof = 0, hif = 0, loo = 0, hio = 0;
        if (mode == ORC_LOD_CAMERA) bounds(d, L, l, 0, &lof, &hif);
        if (mode == ORC_CHUNKED) {
            bounds(d, L, l, offsets[f], &lof, &hif);
            if (o >= 0) bounds(d, L, l, offsets[o], &loo, &hio);
        }
        for (int64_t i = 0; i < lv[l].n; i++) {
            real mu[3] = {lv[l].mean[i], lv[l].mean[lv[l].n + i], lv[l].mean[2 * lv[l].n + i]};
            int in = 0;
            real wi = 1;
            if (mode == ORC_ALL) {
                in = 1;
            } else if (mode == ORC_LOD_CAMERA) {
                real d2 = dist2(mu, pos);
                in = (lof <= d2) && (d2 < hif);
            } else {
                real d2f = dist2(mu, centers + 3 * f);
                int inf_ = (lof <= d2f) && (d2f < hif);
                int ino = 0;
                if (o >= 0) {
                    real d2o = dist2(mu, centers + 3 * o);
                    ino = (loo <= d2o) && (d2o < hio);
                }
                in = inf_ || ino;
                wi = (inf_ && ino) ? (real)1 : (inf_ ? t : t_o);
                if (o < 0) wi = 1;
            }
            if (in) {
                if (count < cap) {
                    ids[count] = (uint32_t)(base + i);
                    w[count] = wi;
                }
                count++;
            }
        }
        base += lv[l].n;
    }
    return count;
}

/* The stored active set of chunk k alone (Sec. 3 "Reducing memory with
 * chunk-based rendering": Eq. 2 evaluated at the chunk centre m_k, every
 * switch distance offset by the chunk's r_k), weight 1 for every member.
 * This is the set the per-chunk visibility filtering renders and prunes.
 * Writes min(count, cap) entries; returns count (-1 on bad arguments). */
int64_t orc_select_chunk(const orc_level* lv, int32_t L, const real* d, const real* centers, const real* offsets,
                         int32_t K, int32_t k, uint32_t* ids, real* w, int64_t cap)
{
    if (k < 0 || k >= K) return -1;
    int64_t count = 0, base = 0;
    for (int32_t l = 0; l < L; l++) {
        real lo, hi;
        bounds(d, L, l, offsets[k], &lo, &hi);
        for (int64_t i = 0; i < lv[l].n; i++) {
            real mu[3] = {lv[l].mean[i], lv[l].mean[lv[l].n + i], lv[l].mean[2 * lv[l].n + i]};
            real d2 = dist2(mu, centers + 3 * k);
            if (lo <= d2 && d2 < hi) {
                if (count < cap) {
                    ids[count] = (uint32_t)(base + i);
                    w[count] = 1;
                }
                count++;
            }
        }
        base += lv[l].n;
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics to degree 3                                      */
/* ------------------------------------------------------------------------ */

/* Basis Y_k, k = l^2 + l + m, evaluated on a unit direction (x, y, z).
 * Normalisation from Y_lm (orthonormal on the sphere); sign convention: the
 * odd-m-negative-side real forms carry a minus sign, i.e.
 *   k1 = -c1 y, k2 = c1 z, k3 = -c1 x,
 *   k4 = c2a xy, k5 = -c2a yz, k6 = c2b (2z^2 - x^2 - y^2), k7 = -c2a xz,
 *   k8 = c2c (x^2 - y^2),
 *   k9 = -c3a y(3x^2 - y^2), k10 = c3b xyz, k11 = -c3c y(4z^2 - x^2 - y^2),
 *   k12 = c3d z(2z^2 - 3x^2 - 3y^2), k13 = -c3c x(4z^2 - x^2 - y^2),
 *   k14 = c3e z(x^2 - y^2), k15 = -c3a x(x^2 - 3y^2)
 * with c0 = 1/(2 sqrt(pi)), c1 = sqrt(3/(4pi)), c2a = sqrt(15/(4pi)),
 * c2b = sqrt(5/(16pi)), c2c = sqrt(15/(16pi)), c3a = sqrt(35/(32pi)),
 * c3b = sqrt(105/(4pi)), c3c = sqrt(21/(32pi)), c3d = sqrt(7/(16pi)),
 * c3e = sqrt(105/(16pi)).  The constants are computed here from these
 * closed forms in double and rounded once. */
typedef struct { real c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e; } sh_consts;

static sh_consts shc(void)
{
    const double pi = 3.14159265358979323846;
    sh_consts s;
    s.c0 = (real)(0.5 / sqrt(pi));
    s.c1 = (real)sqrt(3.0 / (4.0 * pi));
    s.c2a = (real)sqrt(15.0 / (4.0 * pi));
    s.c2b = (real)sqrt(5.0 / (16.0 * pi));
    s.c2c = (real)sqrt(15.0 / (16.0 * pi));
    s.c3a = (real)sqrt(35.0 / (32.0 * pi));
    s.c3b = (real)sqrt(105.0 / (4.0 * pi));
    s.c3c = (real)sqrt(21.0 / (32.0 * pi));
    s.c3d = (real)sqrt(7.0 / (16.0 * pi));
    s.c3e = (real)sqrt(105.0 / (16.0 * pi));
    return s;
}

void orc_sh_basis(real x, real y, real z, real* Y)
{
    sh_consts s = shc();
    real xx = x * x, yy = y * y, zz = z * z;
    Y[0] = s.c0;
    Y[1] = -(s.c1 * y);
    Y[2] = s.c1 * z;
    Y[3] = -(s.c1 * x);
    Y[4] = s.c2a * (x * y);
    Y[5] = -(s.c2a * (y * z));
    Y[6] = s.c2b * ((2 * zz - xx) - yy);
    Y[7] = -(s.c2a * (x * z));
    Y[8] = s.c2c * (xx - yy);
    Y[9] = -(s.c3a * (y * (3 * xx - yy)));
    Y[10] = s.c3b * ((x * y) * z);
    Y[11] = -(s.c3c * (y * ((4 * zz - xx) - yy)));
    Y[12] = s.c3d * (z * ((2 * zz - 3 * xx) - 3 * yy));
    Y[13] = -(s.c3c * (x * ((4 * zz - xx) - yy)));
    Y[14] = s.c3e * (z * (xx - yy));
    Y[15] = -(s.c3a * (x * (xx - 3 * yy)));
}

/* d Y_k / d(x, y, z) of the polynomials above (not restricted to the sphere) */
static void sh_basis_grad(real x, real y, real z, real dY[NSH][3])
{
    sh_consts s = shc();
    real xx = x * x, yy = y * y, zz = z * z;
    memset(dY, 0, sizeof(real) * NSH * 3);
    dY[1][1] = -s.c1;
    dY[2][2] = s.c1;
    dY[3][0] = -s.c1;
    dY[4][0] = s.c2a * y; dY[4][1] = s.c2a * x;
    dY[5][1] = -s.c2a * z; dY[5][2] = -s.c2a * y;
    dY[6][0] = -2 * s.c2b * x; dY[6][1] = -2 * s.c2b * y; dY[6][2] = 4 * s.c2b * z;
    dY[7][0] = -s.c2a * z; dY[7][2] = -s.c2a * x;
    dY[8][0] = 2 * s.c2c * x; dY[8][1] = -2 * s.c2c * y;
    dY[9][0] = -s.c3a * 6 * x * y; dY[9][1] = -s.c3a * (3 * xx - 3 * yy);
    dY[10][0] = s.c3b * y * z; dY[10][1] = s.c3b * x * z; dY[10][2] = s.c3b * x * y;
    dY[11][0] = 2 * s.c3c * x * y; dY[11][1] = -s.c3c * (4 * zz - xx - 3 * yy); dY[11][2] = -8 * s.c3c * y * z;
    dY[12][0] = -6 * s.c3d * x * z; dY[12][1] = -6 * s.c3d * y * z; dY[12][2] = s.c3d * (6 * zz - 3 * xx - 3 * yy);
    dY[13][0] = -s.c3c * (4 * zz - 3 * xx - yy); dY[13][1] = 2 * s.c3c * x * y; dY[13][2] = -8 * s.c3c * x * z;
    dY[14][0] = 2 * s.c3e * x * z; dY[14][1] = -2 * s.c3e * y * z; dY[14][2] = s.c3e * (xx - yy);
    dY[15][0] = -s.c3a * (3 * xx - 3 * yy); dY[15][1] = 6 * s.c3a * x * y;
}

/* ------------------------------------------------------------------------ */
/* projection (EWA splatting + Eq. 3 3-D filter + 2-D filter + SH colour)    */
/* ------------------------------------------------------------------------ */

static int64_t level_of(const orc_level* lv, int32_t L, uint32_t g, int64_t* i)
{
    int64_t base = 0;
    for (int32_t l = 0; l < L; l++) {
        if ((int64_t)g < base + lv[l].n) { *i = (int64_t)g - base; return l; }
        base += lv[l].n;
    }
    return -1;
}

/* Everything the projection of one Gaussian produces, kept for the adjoint. */
typedef struct {
    int visible;
    real mu[3], s[3], q[4], o, w, var;
    real R[9], v[3], Sig[6]; /* Sigma: 00 01 02 11 12 22 */
    real comp3;
    real tc[3];              /* camera-space mean */
    real rx, ry; int clx, cly;
    real J00, J02, J11, J12, M[6];
    real a0, b, c0, a, c, det0, det, comp2;
    real u, v2, A, B, C, radius;
    int32_t rect[4];
    real dir[3], dnorm, rgb_raw[3], rgb[3], o_eff;
} proj_t;

static void project_one(const orc_level* lv, int64_t i, real w, const orc_camera* cam, real s2d,
                        int32_t compensate, proj_t* P)
{
    const int64_t n = lv->n;
    memset(P, 0, sizeof(*P));
    for (int k = 0; k < 3; k++) { P->mu[k] = lv->mean[k * n + i]; P->s[k] = lv->scale[k * n + i]; }
    for (int k = 0; k < 4; k++) P->q[k] = lv->quat[k * n + i];
    P->o = lv->opacity[i];
    P->w = w;
    P->var = lv->filter3d_var;

    /* rotation from the quaternion (w, x, y, z), used as given */
    real qw = P->q[0], qx = P->q[1], qy = P->q[2], qz = P->q[3];
    real xx = qx * qx, yy = qy * qy, zz = qz * qz;
    real xy = qx * qy, xz = qx * qz, yz = qy * qz;
    real wx = qw * qx, wy = qw * qy, wz = qw * qz;
    real* R = P->R;
    R[0] = 1 - 2 * (yy + zz); R[1] = 2 * (xy - wz);     R[2] = 2 * (xz + wy);
    R[3] = 2 * (xy + wz);     R[4] = 1 - 2 * (xx + zz); R[5] = 2 * (yz - wx);
    R[6] = 2 * (xz - wy);     R[7] = 2 * (yz + wx);     R[8] = 1 - 2 * (xx + yy);

    /* Eq. 3: Sigma + var I = R diag(s^2 + var) R^T; opacity factor
     * sqrt(|Sigma| / |Sigma + var I|) = sqrt(prod s_j^2 / (s_j^2 + var)) */
    for (int j = 0; j < 3; j++) P->v[j] = P->s[j] * P->s[j] + P->var;
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; e++) {
        int a = ia[e], b = ib[e];
        P->Sig[e] = ((R[3 * a + 0] * P->v[0]) * R[3 * b + 0] + (R[3 * a + 1] * P->v[1]) * R[3 * b + 1])
                    + (R[3 * a + 2] * P->v[2]) * R[3 * b + 2];
    }
    P->comp3 = R_SQRT(((P->s[0] * P->s[0] / P->v[0]) * (P->s[1] * P->s[1] / P->v[1]))
                      * (P->s[2] * P->s[2] / P->v[2]));

    /* camera space; near-plane cull (znear is a reading: the paper is silent) */
    const real* W = cam->R;
    for (int r = 0; r < 3; r++)
        P->tc[r] = ((W[3 * r] * P->mu[0] + W[3 * r + 1] * P->mu[1]) + W[3 * r + 2] * P->mu[2]) + cam->t[r];
    real tz = P->tc[2];
    if (!(tz > cam->znear)) return;

    /* projected mean; pixel (px, py) is sampled at (px + 0.5, py + 0.5) */
    real ix = P->tc[0] / tz, iy = P->tc[1] / tz;
    P->u = cam->fx * ix + cam->cx;
    P->v2 = cam->fy * iy + cam->cy;

    /* EWA: Jacobian of the perspective map at the (clamped) mean */
    P->rx = ix; P->ry = iy;
    if (P->rx < -cam->lim_x) { P->rx = -cam->lim_x; P->clx = 1; }
    if (P->rx > cam->lim_x) { P->rx = cam->lim_x; P->clx = 1; }
    if (P->ry < -cam->lim_y) { P->ry = -cam->lim_y; P->cly = 1; }
    if (P->ry > cam->lim_y) { P->ry = cam->lim_y; P->cly = 1; }
    P->J00 = cam->fx / tz;
    P->J02 = -((cam->fx * P->rx) / tz);
    P->J11 = cam->fy / tz;
    P->J12 = -((cam->fy * P->ry) / tz);
    /* M = J W (2x3) */
    for (int j = 0; j < 3; j++) {
        P->M[j] = P->J00 * W[j] + P->J02 * W[6 + j];
        P->M[3 + j] = P->J11 * W[3 + j] + P->J12 * W[6 + j];
    }
    /* Sigma' = M Sigma M^T */
    real S3[9] = {P->Sig[0], P->Sig[1], P->Sig[2], P->Sig[1], P->Sig[3], P->Sig[4], P->Sig[2], P->Sig[4], P->Sig[5]};
    real T[6];
    for (int r = 0; r < 2; r++)
        for (int j = 0; j < 3; j++)
            T[3 * r + j] = (P->M[3 * r] * S3[j] + P->M[3 * r + 1] * S3[3 + j]) + P->M[3 * r + 2] * S3[6 + j];
    P->a0 = (T[0] * P->M[0] + T[1] * P->M[1]) + T[2] * P->M[2];
    P->b = (T[0] * P->M[3] + T[1] * P->M[4]) + T[2] * P->M[5];
    P->c0 = (T[3] * P->M[3] + T[4] * P->M[4]) + T[5] * P->M[5];

    /* 2-D screen-space filter with opacity compensation */
    P->a = P->a0 + s2d;
    P->c = P->c0 + s2d;
    P->det0 = P->a0 * P->c0 - P->b * P->b;
    P->det = P->a * P->c - P->b * P->b;
    if (!(P->det > 0)) return;
    P->comp2 = compensate ? R_SQRT((P->det0 > 0 ? P->det0 : (real)0) / P->det) : (real)1;

    /* conic (inverse 2-D covariance) and a 3-sigma radius from the largest eigenvalue */
    P->A = P->c / P->det;
    P->B = -(P->b / P->det);
    P->C = P->a / P->det;
    real mid = (real)0.5 * (P->a + P->c);
    real disc = mid * mid - P->det;
    real lam = mid + R_SQRT(disc > 0 ? disc : (real)0);
    P->radius = R_CEIL((real)3 * R_SQRT(lam));

    /* tile rectangle [x0, x1) x [y0, y1) of 16x16 tiles */
    int32_t TX = (cam->width + TILE - 1) / TILE, TY = (cam->height + TILE - 1) / TILE;
    real fx0 = R_FLOOR((P->u - P->radius) / (real)TILE), fx1 = R_FLOOR((P->u + P->radius) / (real)TILE) + 1;
    real fy0 = R_FLOOR((P->v2 - P->radius) / (real)TILE), fy1 = R_FLOOR((P->v2 + P->radius) / (real)TILE) + 1;
    real lx = -1, hx = (real)(TX + 1), ly = -1, hy = (real)(TY + 1);
    fx0 = fx0 < lx ? lx : (fx0 > hx ? hx : fx0);
    fx1 = fx1 < lx ? lx : (fx1 > hx ? hx : fx1);
    fy0 = fy0 < ly ? ly : (fy0 > hy ? hy : fy0);
    fy1 = fy1 < ly ? ly : (fy1 > hy ? hy : fy1);
    int32_t x0 = (int32_t)fx0, x1 = (int32_t)fx1, y0 = (int32_t)fy0, y1 = (int32_t)fy1;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > TX) x1 = TX;
    if (y1 > TY) y1 = TY;
    if (x0 >= x1 || y0 >= y1) return;
    P->rect[0] = x0; P->rect[1] = y0; P->rect[2] = x1; P->rect[3] = y1;

    /* view-dependent colour: SH in the direction from the camera centre */
    for (int k = 0; k < 3; k++) P->dir[k] = P->mu[k] - cam->pos[k];
    P->dnorm = R_SQRT((P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1]) + P->dir[2] * P->dir[2]);
    real x = P->dir[0] / P->dnorm, y = P->dir[1] / P->dnorm, z = P->dir[2] / P->dnorm;
    real Y[NSH];
    orc_sh_basis(x, y, z, Y);
    int nb = (lv->sh_degree + 1) * (lv->sh_degree + 1);
    for (int ch = 0; ch < 3; ch++) {
        real acc = 0;
        for (int k = 0; k < nb; k++) acc = acc + lv->sh[(k * 3 + ch) * n + i] * Y[k];
        P->rgb_raw[ch] = acc + (real)0.5;
        P->rgb[ch] = P->rgb_raw[ch] > 0 ? P->rgb_raw[ch] : (real)0;
    }
    /* Eq. 4 weight modulates the opacity, before the alpha clamp */
    P->o_eff = ((P->o * P->w) * P->comp3) * P->comp2;
    P->visible = 1;
}

/* Projects every selected Gaussian (active index a = position in ids).
 * Outputs (indexed by a): depth, uv[2], conic[3] (A, B, C), o_eff, rgb[3],
 * rect[4] (x0, y0, x1, y1), tiles (0 = culled). */
void orc_project(const orc_level* lv, int32_t L, const uint32_t* ids, const real* w, int64_t count,
                 const orc_camera* cam, real s2d, int32_t compensate, real* depth, real* uv, real* conic,
                 real* o_eff, real* rgb, int32_t* rect, uint32_t* tiles, real* radius)
{
    ORC_PARALLEL_FOR
    for (int64_t a = 0; a < count; a++) {
        int64_t i;
        int64_t l = level_of(lv, L, ids[a], &i);
        proj_t P;
        if (l < 0) { memset(&P, 0, sizeof(P)); }
        else project_one(&lv[l], i, w[a], cam, s2d, compensate, &P);
        depth[a] = P.tc[2];
        uv[2 * a] = P.u; uv[2 * a + 1] = P.v2;
        conic[3 * a] = P.A; conic[3 * a + 1] = P.B; conic[3 * a + 2] = P.C;
        o_eff[a] = P.o_eff;
        for (int k = 0; k < 3; k++) rgb[3 * a + k] = P.rgb[k];
        for (int k = 0; k < 4; k++) rect[4 * a + k] = P.rect[k];
        tiles[a] = P.visible ? (uint32_t)((P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1])) : 0u;
        if (radius) radius[a] = P.radius;
        if (!P.visible) { depth[a] = 0; tiles[a] = 0; }
    }
}

/* ------------------------------------------------------------------------ */
/* binning + sort by (tile, depth, active index)                             */
/* ------------------------------------------------------------------------ */

typedef struct { uint32_t tile; uint64_t dkey; uint32_t a; } inst_t;

static uint64_t depth_key(real z)
{
    /* depth > 0 here, so the IEEE bit pattern orders like the value */
    if (IS_F32) { float f = (float)z; uint32_t u; memcpy(&u, &f, 4); return u; }
    double g = (double)z; uint64_t u; memcpy(&u, &g, 8); return u;
}

static int inst_cmp(const void* pa, const void* pb)
{
    const inst_t* x = (const inst_t*)pa;
    const inst_t* y = (const inst_t*)pb;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->dkey != y->dkey) return x->dkey < y->dkey ? -1 : 1;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    return 0;
}

/* One instance per (visible Gaussian, tile of its rectangle), sorted with
 * the C library's qsort by (tile, depth bits, active index): a total order.
 * Writes min(M, cap) sorted instances and per-tile [start, end) ranges;
 * returns M. */
int64_t orc_bin_sort(int64_t count, const real* depth, const int32_t* rect, const uint32_t* tiles,
                     int32_t TX, int32_t TY, uint32_t* out_tile, uint64_t* out_dkey, uint32_t* out_val,
                     int64_t cap, uint32_t* ranges)
{
    int64_t M = 0;
    for (int64_t a = 0; a < count; a++) M += tiles[a];
    inst_t* in = (inst_t*)malloc(sizeof(inst_t) * (size_t)(M > 0 ? M : 1));
    int64_t m = 0;
    for (int64_t a = 0; a < count; a++) {
        if (!tiles[a]) continue;
        for (int32_t ty = rect[4 * a + 1]; ty < rect[4 * a + 3]; ty++)
            for (int32_t tx = rect[4 * a + 0]; tx < rect[4 * a + 2]; tx++) {
                in[m].tile = (uint32_t)(ty * TX + tx);
                in[m].dkey = depth_key(depth[a]);
                in[m].a = (uint32_t)a;
                m++;
            }
    }
    qsort(in, (size_t)M, sizeof(inst_t), inst_cmp);
    for (int64_t t = 0; t < (int64_t)TX * TY; t++) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t k = 0; k < M; k++) {
        uint32_t t = in[k].tile;
        if (k == 0 || in[k - 1].tile != t) ranges[2 * t] = (uint32_t)k;
        ranges[2 * t + 1] = (uint32_t)(k + 1);
        if (k < cap) { out_tile[k] = t; out_dkey[k] = in[k].dkey; out_val[k] = in[k].a; }
    }
    free(in);
    return M;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 + front-to-back alpha compositing of one pixel                      */
/* ------------------------------------------------------------------------ */

/* Thresholds (paper silent; the 3DGS renderer conventions): alpha is
 * clamped to 0.99, entries with alpha < 1/255 are skipped, and a pixel
 * stops, without blending the entry, once T (1 - alpha) < 1e-4. */
#define ALPHA_MAX ((real)0.99)
#define ALPHA_MIN ((real)(1.0f / 255.0f))
#define T_STOP ((real)0.0001f)
/* relative margin inside which a threshold decision may legitimately differ
 * between two correct FP32 renderers whose exp differs by a few ulp */
#define NEAR_REL ((real)1e-5)
#define NEAR_POW ((real)1e-6)

typedef struct {
    real C[3], T;
    uint32_t n_contrib, n_blend, n_eval;
    int near;
    /* flips: decision indices (counted over all threshold decisions) to invert */
    const int* flip; int nflip;
    int ndec;           /* number of near decisions seen */
    int64_t first_near; /* list position of the first near decision (len if none) */
    int dec_near[64];   /* decision indices of near decisions */
    /* optional per-entry trace for the adjoint */
    int64_t cap_trace;  int64_t ntrace;
    int64_t* tr_pos; real* tr_alpha; real* tr_T; int* tr_clamped; real* tr_G;
} pix_t;

static int flipped(const pix_t* S, int dec)
{
    for (int k = 0; k < S->nflip; k++) if (S->flip[k] == dec) return 1;
    return 0;
}

/* list[k] (k < len) are active indices in blend order */
static void composite_pixel(const uint32_t* list, int64_t len, real px, real py, const real* uv, const real* conic,
                            const real* o_eff, const real* rgb, pix_t* S)
{
    S->C[0] = S->C[1] = S->C[2] = 0;
    S->T = 1;
    S->n_contrib = 0; S->n_blend = 0; S->n_eval = 0; S->near = 0; S->ndec = 0; S->ntrace = 0;
    S->first_near = len;
    int dec = 0;
    for (int64_t k = 0; k < len; k++) {
        uint32_t a = list[k];
        S->n_eval = (uint32_t)(k + 1);
        real dx = uv[2 * a] - px, dy = uv[2 * a + 1] - py;
        real A = conic[3 * a], B = conic[3 * a + 1], C = conic[3 * a + 2];
        real power = (real)-0.5 * ((A * dx) * dx + (C * dy) * dy) - (B * dx) * dy;
        int skip = power > 0;
        if ((power > 0 ? power : -power) < NEAR_POW) { if (S->ndec < 64) S->dec_near[S->ndec++] = dec; if (!S->near) S->first_near = k; S->near = 1; }
        if (flipped(S, dec)) skip = !skip;
        dec++;
        if (skip) continue;
        real G = R_EXP(power);
        real og = o_eff[a] * G;
        real alpha = og < ALPHA_MAX ? og : ALPHA_MAX;
        int lowa = alpha < ALPHA_MIN;
        real da = alpha - ALPHA_MIN;
        if ((da > 0 ? da : -da) <= NEAR_REL * ALPHA_MIN) { if (S->ndec < 64) S->dec_near[S->ndec++] = dec; if (!S->near) S->first_near = k; S->near = 1; }
        if (flipped(S, dec)) lowa = !lowa;
        dec++;
        if (lowa) continue;
        real Tn = S->T * ((real)1 - alpha);
        int stop = Tn < T_STOP;
        real dt = Tn - T_STOP;
        if ((dt > 0 ? dt : -dt) <= NEAR_REL * T_STOP) { if (S->ndec < 64) S->dec_near[S->ndec++] = dec; if (!S->near) S->first_near = k; S->near = 1; }
        if (flipped(S, dec)) stop = !stop;
        dec++;
        if (stop) break;
        if (S->ntrace < S->cap_trace) {
            S->tr_pos[S->ntrace] = k;
            S->tr_alpha[S->ntrace] = alpha;
            S->tr_T[S->ntrace] = S->T;
            S->tr_clamped[S->ntrace] = !(og < ALPHA_MAX);
            S->tr_G[S->ntrace] = G;
        }
        S->ntrace++;
        for (int ch = 0; ch < 3; ch++) S->C[ch] = S->C[ch] + rgb[3 * a + ch] * (alpha * S->T);
        S->T = Tn;
        S->n_contrib = (uint32_t)(k + 1);
        S->n_blend++;
    }
}

/* Tiled compositor: each pixel walks its tile's sorted list.
 * Outputs image[3][H][W] = C + T bg, final_T[H][W], n_contrib[H][W]
 * (position + 1 of the last blended list entry), and optional per-pixel
 * n_blend, n_eval (entries evaluated until termination) and near flags. */
void orc_composite(const orc_camera* cam, const real* uv, const real* conic, const real* o_eff, const real* rgb,
                   const uint32_t* ranges, const uint32_t* vals, real* image, real* final_T, uint32_t* n_contrib,
                   uint32_t* n_blend, uint32_t* n_eval, uint8_t* near)
{
    int32_t W = cam->width, H = cam->height, TX = (W + TILE - 1) / TILE;
    ORC_PARALLEL_ROWS
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t t = (y / TILE) * TX + (x / TILE);
            pix_t S; memset(&S, 0, sizeof(S));
            composite_pixel(vals + ranges[2 * t], (int64_t)ranges[2 * t + 1] - ranges[2 * t], (real)x + (real)0.5,
                            (real)y + (real)0.5, uv, conic, o_eff, rgb, &S);
            int64_t p = (int64_t)y * W + x;
            for (int ch = 0; ch < 3; ch++) image[(int64_t)ch * H * W + p] = S.C[ch] + S.T * cam->bg[ch];
            final_T[p] = S.T;
            n_contrib[p] = S.n_contrib;
            if (n_blend) n_blend[p] = S.n_blend;
            if (n_eval) n_eval[p] = S.n_eval;
            if (near) near[p] = (uint8_t)S.near;
        }
}

/* The same per-pixel walk for listed pixels only (x[k], y[k]): colour
 * rgb[k][3] = C + T bg, final_T[k], n_contrib[k], near[k].  Used to check
 * sampled pixels of full-size frames. */
void orc_composite_pixels(const orc_camera* cam, const real* uv, const real* conic, const real* o_eff,
                          const real* rgb, const uint32_t* ranges, const uint32_t* vals, int64_t n,
                          const int32_t* xs, const int32_t* ys, real* color, real* final_T, uint32_t* n_contrib,
                          uint8_t* near)
{
    int32_t TX = (cam->width + TILE - 1) / TILE;
    for (int64_t k = 0; k < n; k++) {
        int32_t x = xs[k], y = ys[k];
        int32_t t = (y / TILE) * TX + (x / TILE);
        pix_t S; memset(&S, 0, sizeof(S));
        composite_pixel(vals + ranges[2 * t], (int64_t)ranges[2 * t + 1] - ranges[2 * t], (real)x + (real)0.5,
                        (real)y + (real)0.5, uv, conic, o_eff, rgb, &S);
        for (int ch = 0; ch < 3; ch++) color[3 * k + ch] = S.C[ch] + S.T * cam->bg[ch];
        final_T[k] = S.T;
        n_contrib[k] = S.n_contrib;
        near[k] = (uint8_t)S.near;
    }
}

/* Brute-force compositor: for each pixel, every visible Gaussian whose tile
 * rectangle contains the pixel's tile, sorted by (depth bits, active index)
 * on the spot.  Independent of the binning and the sort above. */
static uint64_t* g_bf_keys_d;
static int bf_cmp(const void* pa, const void* pb)
{
    int64_t x = *(const int64_t*)pa, y = *(const int64_t*)pb;
    if (g_bf_keys_d[x] != g_bf_keys_d[y]) return g_bf_keys_d[x] < g_bf_keys_d[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

void orc_composite_brute(const orc_camera* cam, int64_t count, const real* depth, const int32_t* rect,
                         const uint32_t* tiles, const real* uv, const real* conic, const real* o_eff,
                         const real* rgb, real* image, real* final_T, uint32_t* n_contrib)
{
    int32_t W = cam->width, H = cam->height;
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    uint32_t* list = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(count > 0 ? count : 1));
    uint64_t* dk = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(count > 0 ? count : 1));
    for (int64_t a = 0; a < count; a++) dk[a] = depth_key(depth[a]);
    g_bf_keys_d = dk;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t tx = x / TILE, ty = y / TILE;
            int64_t m = 0;
            for (int64_t a = 0; a < count; a++)
                if (tiles[a] && rect[4 * a] <= tx && tx < rect[4 * a + 2] && rect[4 * a + 1] <= ty && ty < rect[4 * a + 3])
                    idx[m++] = a;
            qsort(idx, (size_t)m, sizeof(int64_t), bf_cmp);
            for (int64_t k = 0; k < m; k++) list[k] = (uint32_t)idx[k];
            pix_t S; memset(&S, 0, sizeof(S));
            composite_pixel(list, m, (real)x + (real)0.5, (real)y + (real)0.5, uv, conic, o_eff, rgb, &S);
            int64_t p = (int64_t)y * W + x;
            for (int ch = 0; ch < 3; ch++) image[(int64_t)ch * H * W + p] = S.C[ch] + S.T * cam->bg[ch];
            final_T[p] = S.T;
            n_contrib[p] = S.n_contrib;
        }
    free(idx); free(list); free(dk);
}

/* Composites pixel (x, y) of the tiled lists with up to two near-threshold
 * decisions inverted and reports whether any such variant (or the plain
 * trace) lands within tol of `probe` on every channel.  Used to accept a
 * pixel where two correct renderers branch differently on a threshold. */
int orc_pixel_accept(const orc_camera* cam, const real* uv, const real* conic, const real* o_eff, const real* rgb,
                     const uint32_t* ranges, const uint32_t* vals, int32_t x, int32_t y, const real* probe, real tol)
{
    int32_t TX = (cam->width + TILE - 1) / TILE;
    int32_t t = (y / TILE) * TX + (x / TILE);
    const uint32_t* list = vals + ranges[2 * t];
    int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
    real px = (real)x + (real)0.5, py = (real)y + (real)0.5;
    pix_t S; memset(&S, 0, sizeof(S));
    composite_pixel(list, len, px, py, uv, conic, o_eff, rgb, &S);
    int nd = S.ndec;
    int decs[64];
    memcpy(decs, S.dec_near, sizeof(int) * (size_t)nd);
#define ACCEPTS(SS) (fabs((double)((SS).C[0] + (SS).T * cam->bg[0] - probe[0])) <= (double)tol && \
                     fabs((double)((SS).C[1] + (SS).T * cam->bg[1] - probe[1])) <= (double)tol && \
                     fabs((double)((SS).C[2] + (SS).T * cam->bg[2] - probe[2])) <= (double)tol)
    if (ACCEPTS(S)) return 1;
    for (int i = 0; i < nd; i++) {
        int fl[2] = {decs[i], 0};
        pix_t V; memset(&V, 0, sizeof(V)); V.flip = fl; V.nflip = 1;
        composite_pixel(list, len, px, py, uv, conic, o_eff, rgb, &V);
        if (ACCEPTS(V)) return 1;
        /* a flip can expose a later near decision: try it paired */
        for (int j = 0; j < V.ndec; j++) {
            if (V.dec_near[j] == decs[i]) continue;
            int fl2[2] = {decs[i], V.dec_near[j]};
            pix_t V2; memset(&V2, 0, sizeof(V2)); V2.flip = fl2; V2.nflip = 2;
            composite_pixel(list, len, px, py, uv, conic, o_eff, rgb, &V2);
            if (ACCEPTS(V2)) return 1;
        }
    }
#undef ACCEPTS
    return 0;
}

/* ------------------------------------------------------------------------ */
/* importance scores (Sec. 3 "Preliminaries: Importance pruning",            */
/* "Visibility filtering")                                                   */
/* ------------------------------------------------------------------------ */

/* The importance of a Gaussian is the largest blending weight it receives
 * in any pixel of any view: for an entry blended at a pixel, alpha times
 * the transmittance in front of it (its contribution to the pixel colour
 * per unit colour).  Entries that are skipped (alpha < 1/255) or that stop
 * the pixel contribute nothing and have weight 0.
 *
 * For one view (its tiled lists): every pixel walks its list as the
 * compositor does, and score[ids[a]] = max(score[ids[a]], alpha T) over its
 * blended entries a.  score is indexed by global id and max-accumulated, so
 * calls over several views give the maximum over all of them (the caller
 * starts it at 0).  amb (optional, by global id, OR-accumulated) marks the
 * Gaussians listed at or after the first near-threshold decision of some
 * pixel: there a correct FP32 renderer may branch the other way, and the
 * Gaussian's weight in that pixel is not fixed to rounding. */
void orc_importance(const orc_camera* cam, const real* uv, const real* conic, const real* o_eff, const real* rgb,
                    const uint32_t* ranges, const uint32_t* vals, const uint32_t* ids, real* score, uint8_t* amb)
{
    int32_t W = cam->width, H = cam->height, TX = (W + TILE - 1) / TILE, TY = (H + TILE - 1) / TILE;
    int64_t maxlen = 1;
    for (int32_t t = 0; t < TX * TY; t++) {
        int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
        if (len > maxlen) maxlen = len;
    }
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)maxlen);
    real* ta = (real*)malloc(sizeof(real) * (size_t)maxlen);
    real* tT = (real*)malloc(sizeof(real) * (size_t)maxlen);
    int* tc = (int*)malloc(sizeof(int) * (size_t)maxlen);
    real* tG = (real*)malloc(sizeof(real) * (size_t)maxlen);
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t t = (y / TILE) * TX + (x / TILE);
            const uint32_t* list = vals + ranges[2 * t];
            int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
            pix_t S; memset(&S, 0, sizeof(S));
            S.cap_trace = maxlen; S.tr_pos = pos; S.tr_alpha = ta; S.tr_T = tT; S.tr_clamped = tc; S.tr_G = tG;
            composite_pixel(list, len, (real)x + (real)0.5, (real)y + (real)0.5, uv, conic, o_eff, rgb, &S);
            for (int64_t j = 0; j < S.ntrace; j++) {
                uint32_t g = ids[list[pos[j]]];
                real wgt = ta[j] * tT[j];
                if (wgt > score[g]) score[g] = wgt;
            }
            if (amb)
                for (int64_t k = S.first_near; k < len; k++) amb[ids[list[k]]] = 1;
        }
    free(pos); free(ta); free(tT); free(tc); free(tG);
}

/* The blending weights of one pixel (x, y) of the tiled lists: for each of
 * its blended entries, in blend order, the active index and alpha T; at most
 * cap of them are written; returns their number (-1 if cap is too small).
 * *near_pos receives the list position of the pixel's first near-threshold
 * decision (the list length if none).  Used to check importance scores of
 * full-size frames at sampled pixels. */
int64_t orc_pixel_weights(const orc_camera* cam, const real* uv, const real* conic, const real* o_eff, const real* rgb,
                          const uint32_t* ranges, const uint32_t* vals, int32_t x, int32_t y, uint32_t* act,
                          real* weight, int64_t* pos, int64_t cap, int64_t* near_pos)
{
    int32_t TX = (cam->width + TILE - 1) / TILE;
    int32_t t = (y / TILE) * TX + (x / TILE);
    const uint32_t* list = vals + ranges[2 * t];
    int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
    int64_t n = len > 0 ? len : 1;
    int64_t* tp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    real* ta = (real*)malloc(sizeof(real) * (size_t)n);
    real* tT = (real*)malloc(sizeof(real) * (size_t)n);
    int* tc = (int*)malloc(sizeof(int) * (size_t)n);
    real* tG = (real*)malloc(sizeof(real) * (size_t)n);
    pix_t S; memset(&S, 0, sizeof(S));
    S.cap_trace = n; S.tr_pos = tp; S.tr_alpha = ta; S.tr_T = tT; S.tr_clamped = tc; S.tr_G = tG;
    composite_pixel(list, len, (real)x + (real)0.5, (real)y + (real)0.5, uv, conic, o_eff, rgb, &S);
    int64_t m = S.ntrace;
    if (m <= cap)
        for (int64_t j = 0; j < m; j++) {
            act[j] = list[tp[j]];
            weight[j] = ta[j] * tT[j];
            pos[j] = tp[j];
        }
    *near_pos = S.first_near;
    free(tp); free(ta); free(tT); free(tc); free(tG);
    return m <= cap ? m : -1;
}

/* ------------------------------------------------------------------------ */
/* adjoint (reverse mode by hand), used in the FP64 build                    */
/* ------------------------------------------------------------------------ */

/* Gradients of L = sum dL_dimage * image with respect to the 2-D quantities
 * of each active Gaussian: g2[a*9 + {u, v, A, B, C, o_eff, r, g, b}] (+=).
 * Each pixel's forward trace is recomputed and walked back to front:
 *   dC/dc_k = alpha_k T_k,
 *   dC/dalpha_k = c_k T_k - S_k / (1 - alpha_k),
 * with S_k = sum_{j>k} c_j alpha_j T_j + T_final bg.  The alpha clamp and the
 * rgb clamp give zero gradient where active. */
void orc_composite_grad2d(const orc_camera* cam, const real* uv, const real* conic, const real* o_eff,
                          const real* rgb, const uint32_t* ranges, const uint32_t* vals, const real* dL_dimage,
                          real* g2)
{
    int32_t W = cam->width, H = cam->height, TX = (W + TILE - 1) / TILE;
    int64_t maxlen = 1;
    for (int64_t t = 0; t < (int64_t)TX * ((H + TILE - 1) / TILE); t++) {
        int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
        if (len > maxlen) maxlen = len;
    }
    int64_t* tr_pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)maxlen);
    real* tr_alpha = (real*)malloc(sizeof(real) * (size_t)maxlen);
    real* tr_T = (real*)malloc(sizeof(real) * (size_t)maxlen);
    int* tr_cl = (int*)malloc(sizeof(int) * (size_t)maxlen);
    real* tr_G = (real*)malloc(sizeof(real) * (size_t)maxlen);
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int64_t p = (int64_t)y * W + x;
            /* a pixel whose loss gradient is zero adds nothing to any gradient */
            if (dL_dimage[p] == 0 && dL_dimage[(int64_t)H * W + p] == 0 && dL_dimage[2 * (int64_t)H * W + p] == 0)
                continue;
            int32_t t = (y / TILE) * TX + (x / TILE);
            const uint32_t* list = vals + ranges[2 * t];
            int64_t len = (int64_t)ranges[2 * t + 1] - ranges[2 * t];
            real px = (real)x + (real)0.5, py = (real)y + (real)0.5;
            pix_t S; memset(&S, 0, sizeof(S));
            S.cap_trace = maxlen; S.tr_pos = tr_pos; S.tr_alpha = tr_alpha; S.tr_T = tr_T; S.tr_clamped = tr_cl;
            S.tr_G = tr_G;
            composite_pixel(list, len, px, py, uv, conic, o_eff, rgb, &S);
            real dC[3];
            for (int ch = 0; ch < 3; ch++) dC[ch] = dL_dimage[(int64_t)ch * H * W + p];
            real Sfx[3];
            for (int ch = 0; ch < 3; ch++) Sfx[ch] = S.T * cam->bg[ch];
            for (int64_t k = S.ntrace - 1; k >= 0; k--) {
                uint32_t a = list[tr_pos[k]];
                real al = tr_alpha[k], Tk = tr_T[k];
                real* g = g2 + 9 * (int64_t)a;
                real dal = 0;
                for (int ch = 0; ch < 3; ch++) {
                    real c = rgb[3 * a + ch];
                    g[6 + ch] += al * Tk * dC[ch];
                    dal += dC[ch] * (c * Tk - Sfx[ch] / ((real)1 - al));
                    Sfx[ch] += c * al * Tk;
                }
                if (tr_cl[k]) continue;
                real G = tr_G[k];
                real o = o_eff[a];
                g[5] += dal * G;
                real dpow = dal * o * G;
                real dx = uv[2 * a] - px, dy = uv[2 * a + 1] - py;
                real A = conic[3 * a], B = conic[3 * a + 1], Cc = conic[3 * a + 2];
                g[2] += (real)-0.5 * dx * dx * dpow;
                g[3] += -dx * dy * dpow;
                g[4] += (real)-0.5 * dy * dy * dpow;
                g[0] += (-A * dx - B * dy) * dpow;
                g[1] += (-Cc * dy - B * dx) * dpow;
            }
        }
    free(tr_pos); free(tr_alpha); free(tr_T); free(tr_cl); free(tr_G);
}

/* Chains the 2-D gradients of each visible active Gaussian back to its
 * activated parameters (mean, scale, quaternion as given, opacity, SH) and
 * adds them to grads[level].  grad_level >= 0 restricts the update to that
 * level's Gaussians (the per-level fine-tuning updates only G_l). */
void orc_project_grad(const orc_level* lv, int32_t L, const uint32_t* ids, const real* w, int64_t count,
                      const orc_camera* cam, real s2d, int32_t compensate, const real* g2, int32_t grad_level,
                      orc_grads* grads)
{
    for (int64_t a = 0; a < count; a++) {
        int64_t i;
        int64_t l = level_of(lv, L, ids[a], &i);
        if (l < 0) continue;
        if (grad_level >= 0 && l != grad_level) continue;
        proj_t P;
        project_one(&lv[l], i, w[a], cam, s2d, compensate, &P);
        if (!P.visible) continue;
        const real* g = g2 + 9 * a;
        const int64_t n = lv[l].n;
        orc_grads* G = &grads[l];
        real dmu[3] = {0, 0, 0}, ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0};

        /* colour: rgb = max(0, sum_k sh_k Y_k(dir) + 0.5), dir = (mu - pos)/|mu - pos| */
        real x = P.dir[0] / P.dnorm, y = P.dir[1] / P.dnorm, z = P.dir[2] / P.dnorm;
        real Y[NSH], dY[NSH][3];
        orc_sh_basis(x, y, z, Y);
        sh_basis_grad(x, y, z, dY);
        int nb = (lv[l].sh_degree + 1) * (lv[l].sh_degree + 1);
        real ddir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            if (!(P.rgb_raw[ch] > 0)) continue;
            real gc = g[6 + ch];
            for (int k = 0; k < nb; k++) {
                G->sh[(k * 3 + ch) * n + i] += gc * Y[k];
                real shk = lv[l].sh[(k * 3 + ch) * n + i];
                for (int j = 0; j < 3; j++) ddir[j] += gc * shk * dY[k][j];
            }
        }
        real dn[3] = {x, y, z};
        real dot = ddir[0] * dn[0] + ddir[1] * dn[1] + ddir[2] * dn[2];
        for (int j = 0; j < 3; j++) dmu[j] += (ddir[j] - dn[j] * dot) / P.dnorm;

        /* opacity: o_eff = o w comp3 comp2 */
        real go = g[5];
        G->opacity[i] += go * P.w * P.comp3 * P.comp2;
        real dcomp3 = go * P.o * P.w * P.comp2;
        real dcomp2 = go * P.o * P.w * P.comp3;

        /* conic (A, B, C) = (c, -b, a) / det with a = a0 + s2d, c = c0 + s2d */
        real det = P.det, det2 = det * det;
        real ga = 0, gb = 0, gc_ = 0;
        ga += g[2] * (-(P.c * P.c) / det2) + g[3] * (P.b * P.c / det2) + g[4] * (-(P.b * P.b) / det2);
        gc_ += g[2] * (-(P.b * P.b) / det2) + g[3] * (P.b * P.a / det2) + g[4] * (-(P.a * P.a) / det2);
        gb += g[2] * (2 * P.b * P.c / det2) + g[3] * (-(P.a * P.c + P.b * P.b) / det2) + g[4] * (2 * P.a * P.b / det2);
        /* comp2 = sqrt(det0 / det) */
        if (compensate && P.det0 > 0) {
            real ddet0 = dcomp2 / (2 * P.comp2 * det);
            real ddet = -dcomp2 * P.comp2 / (2 * det);
            ga += ddet0 * P.c0 + ddet * P.c;
            gc_ += ddet0 * P.a0 + ddet * P.a;
            gb += ddet0 * (-2 * P.b) + ddet * (-2 * P.b);
        }
        /* Sigma' = M Sigma M^T: dL/dSigma = M^T G' M, dL/dM = 2 G' M Sigma, G' = [[ga, gb/2], [gb/2, gc]] */
        real Gp[4] = {ga, gb / 2, gb / 2, gc_};
        const real* M = P.M;
        real S3[9] = {P.Sig[0], P.Sig[1], P.Sig[2], P.Sig[1], P.Sig[3], P.Sig[4], P.Sig[2], P.Sig[4], P.Sig[5]};
        real dSig[9];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                real acc = 0;
                for (int p = 0; p < 2; p++)
                    for (int q = 0; q < 2; q++) acc += M[3 * p + r] * Gp[2 * p + q] * M[3 * q + c];
                dSig[3 * r + c] = acc;
            }
        real dM[6];
        for (int p = 0; p < 2; p++)
            for (int c = 0; c < 3; c++) {
                real acc = 0;
                for (int q = 0; q < 2; q++)
                    for (int k = 0; k < 3; k++) acc += 2 * Gp[2 * p + q] * M[3 * q + k] * S3[3 * k + c];
                dM[3 * p + c] = acc;
            }
        /* M = J W: dJ = dM W^T (only the four non-zero entries of J matter) */
        const real* Wc = cam->R;
        real dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
        for (int c = 0; c < 3; c++) {
            dJ00 += dM[c] * Wc[c];
            dJ02 += dM[c] * Wc[6 + c];
            dJ11 += dM[3 + c] * Wc[3 + c];
            dJ12 += dM[3 + c] * Wc[6 + c];
        }
        /* J entries and the projected mean as functions of the camera-space mean */
        real tx = P.tc[0], ty = P.tc[1], tz = P.tc[2];
        real dtc[3] = {0, 0, 0};
        dtc[2] += dJ00 * (-cam->fx / (tz * tz)) + dJ11 * (-cam->fy / (tz * tz));
        if (P.clx) dtc[2] += dJ02 * (cam->fx * P.rx / (tz * tz));
        else { dtc[0] += dJ02 * (-cam->fx / (tz * tz)); dtc[2] += dJ02 * (2 * cam->fx * tx / (tz * tz * tz)); }
        if (P.cly) dtc[2] += dJ12 * (cam->fy * P.ry / (tz * tz));
        else { dtc[1] += dJ12 * (-cam->fy / (tz * tz)); dtc[2] += dJ12 * (2 * cam->fy * ty / (tz * tz * tz)); }
        dtc[0] += g[0] * cam->fx / tz;
        dtc[2] += g[0] * (-cam->fx * tx / (tz * tz));
        dtc[1] += g[1] * cam->fy / tz;
        dtc[2] += g[1] * (-cam->fy * ty / (tz * tz));
        for (int j = 0; j < 3; j++) dmu[j] += Wc[j] * dtc[0] + Wc[3 + j] * dtc[1] + Wc[6 + j] * dtc[2];

        /* Sigma = R diag(v) R^T: dv_j = (R^T dSig R)_jj, dR = 2 dSig R diag(v) */
        const real* R = P.R;
        real dv[3], dR[9];
        for (int j = 0; j < 3; j++) {
            real acc = 0;
            for (int a2 = 0; a2 < 3; a2++)
                for (int b2 = 0; b2 < 3; b2++) acc += R[3 * a2 + j] * dSig[3 * a2 + b2] * R[3 * b2 + j];
            dv[j] = acc;
        }
        for (int a2 = 0; a2 < 3; a2++)
            for (int j = 0; j < 3; j++) {
                real acc = 0;
                for (int b2 = 0; b2 < 3; b2++) acc += dSig[3 * a2 + b2] * R[3 * b2 + j];
                dR[3 * a2 + j] = 2 * acc * P.v[j];
            }
        /* v_j = s_j^2 + var; comp3 = sqrt(prod s_j^2 / v_j) -> d comp3 / d s_j = comp3 var / (s_j v_j) */
        for (int j = 0; j < 3; j++) {
            ds[j] += dv[j] * 2 * P.s[j];
            ds[j] += dcomp3 * P.comp3 * P.var / (P.s[j] * P.v[j]);
        }
        /* R(q) */
        real qw = P.q[0], qx = P.q[1], qy = P.q[2], qz = P.q[3];
        dq[0] += dR[1] * (-2 * qz) + dR[2] * (2 * qy) + dR[3] * (2 * qz) + dR[5] * (-2 * qx) + dR[6] * (-2 * qy)
                 + dR[7] * (2 * qx);
        dq[1] += dR[1] * (2 * qy) + dR[2] * (2 * qz) + dR[3] * (2 * qy) + dR[4] * (-4 * qx) + dR[5] * (-2 * qw)
                 + dR[6] * (2 * qz) + dR[7] * (2 * qw) + dR[8] * (-4 * qx);
        dq[2] += dR[0] * (-4 * qy) + dR[1] * (2 * qx) + dR[2] * (2 * qw) + dR[3] * (2 * qx) + dR[5] * (2 * qz)
                 + dR[6] * (-2 * qw) + dR[7] * (2 * qz) + dR[8] * (-4 * qy);
        dq[3] += dR[0] * (-4 * qz) + dR[1] * (-2 * qw) + dR[2] * (2 * qx) + dR[3] * (2 * qw) + dR[4] * (-4 * qz)
                 + dR[5] * (2 * qy) + dR[6] * (2 * qx) + dR[7] * (2 * qy);

        for (int j = 0; j < 3; j++) { G->mean[j * n + i] += dmu[j]; G->scale[j * n + i] += ds[j]; }
        for (int j = 0; j < 4; j++) G->quat[j * n + i] += dq[j];
    }
}
