/*
 * TEST INFRASTRUCTURE ONLY: a driver that runs every step of the oracle on
 * a small scene, for builds with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py builds it
 * with each of REAL=float and REAL=double, linked with lodge_oracle.c).
 * It makes its own inputs (a fixed linear congruential generator), and
 * besides exercising every entry point it checks the one identity the
 * oracle owes itself here: the tiled compositor equals the brute-force one
 * bit for bit.  Exit status 0: every step ran clean.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL float
#endif
typedef REAL real;

/* the oracle's inputs, as it declares them */
typedef struct {
    int64_t n;
    const real *mean, *scale, *quat, *opacity, *sh;
    int32_t sh_degree;
    real filter3d_var;
} orc_level;
typedef struct {
    int32_t width, height;
    real fx, fy, cx, cy;
    real R[9], t[3], pos[3];
    real znear, lim_x, lim_y;
    real bg[3];
} orc_camera;
typedef struct {
    real *mean, *scale, *quat, *opacity, *sh;
} orc_grads;

int orc_chunk_pair(const real*, int32_t, real, const real*, int32_t*, int32_t*, real*);
int64_t orc_select(const orc_level*, int32_t, const real*, int32_t, const real*, const real*, int32_t, real,
                   const real*, uint32_t*, real*, int64_t, int32_t*, int32_t*, real*);
int64_t orc_select_chunk(const orc_level*, int32_t, const real*, const real*, const real*, int32_t, int32_t,
                         uint32_t*, real*, int64_t);
void orc_project(const orc_level*, int32_t, const uint32_t*, const real*, int64_t, const orc_camera*, real,
                 int32_t, real*, real*, real*, real*, real*, int32_t*, uint32_t*, real*);
int64_t orc_bin_sort(int64_t, const real*, const int32_t*, const uint32_t*, int32_t, int32_t, uint32_t*,
                     uint64_t*, uint32_t*, int64_t, uint32_t*);
void orc_composite(const orc_camera*, const real*, const real*, const real*, const real*, const uint32_t*,
                   const uint32_t*, real*, real*, uint32_t*, uint32_t*, uint32_t*, uint8_t*);
void orc_composite_pixels(const orc_camera*, const real*, const real*, const real*, const real*, const uint32_t*,
                          const uint32_t*, int64_t, const int32_t*, const int32_t*, real*, real*, uint32_t*,
                          uint8_t*);
void orc_composite_brute(const orc_camera*, int64_t, const real*, const int32_t*, const uint32_t*, const real*,
                         const real*, const real*, const real*, real*, real*, uint32_t*);
int orc_pixel_accept(const orc_camera*, const real*, const real*, const real*, const real*, const uint32_t*,
                     const uint32_t*, int32_t, int32_t, const real*, real);
void orc_importance(const orc_camera*, const real*, const real*, const real*, const real*, const uint32_t*,
                    const uint32_t*, const uint32_t*, real*, uint8_t*);
int64_t orc_pixel_weights(const orc_camera*, const real*, const real*, const real*, const real*, const uint32_t*,
                          const uint32_t*, int32_t, int32_t, uint32_t*, real*, int64_t*, int64_t, int64_t*);
void orc_composite_grad2d(const orc_camera*, const real*, const real*, const real*, const real*, const uint32_t*,
                          const uint32_t*, const real*, real*);
void orc_project_grad(const orc_level*, int32_t, const uint32_t*, const real*, int64_t, const orc_camera*, real,
                      int32_t, const real*, int32_t, orc_grads*);
void orc_sh_basis(real, real, real, real*);

static uint64_t lcg_state = 0x2505231580ull;
static double uni(void)   /* uniform in [0, 1) */
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static void* must(size_t bytes)
{
    void* p = calloc(1, bytes > 0 ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

#define FAIL(...) do { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); return 1; } while (0)

int main(void)
{
    enum { L = 2, K = 4, W = 40, H = 36, TILE = 16 };
    const int64_t n[L] = {300, 90};
    orc_level lv[L];
    real* planes[L][5];
    for (int l = 0; l < L; l++) {
        const int64_t m = n[l];
        real* mean = must(sizeof(real) * 3 * m);
        real* scale = must(sizeof(real) * 3 * m);
        real* quat = must(sizeof(real) * 4 * m);
        real* opacity = must(sizeof(real) * m);
        real* sh = must(sizeof(real) * 48 * m);
        for (int64_t i = 0; i < 3 * m; i++) mean[i] = (real)(4.0 * uni() - 2.0);
        for (int64_t i = 0; i < 3 * m; i++) scale[i] = (real)exp(-2.5 + 0.6 * uni() + 0.7 * l);
        for (int64_t i = 0; i < m; i++) {
            double q[4], s = 0.0;
            for (int c = 0; c < 4; c++) { q[c] = uni() - 0.5; s += q[c] * q[c]; }
            for (int c = 0; c < 4; c++) quat[c * m + i] = (real)(q[c] / sqrt(s));
            opacity[i] = (real)(0.05 + 0.9 * uni());
        }
        for (int64_t i = 0; i < 48 * m; i++) sh[i] = (real)(i < 3 * m ? 0.5 + 0.2 * (uni() - 0.5) : 0.1 * (uni() - 0.5));
        lv[l] = (orc_level){m, mean, scale, quat, opacity, sh, 3, (real)(l == 0 ? 0.0 : 0.002)};
        planes[l][0] = mean; planes[l][1] = scale; planes[l][2] = quat; planes[l][3] = opacity; planes[l][4] = sh;
    }
    const real d[1] = {(real)5.5};
    real centers[3 * K], offsets[K];
    for (int k = 0; k < K; k++) {
        centers[3 * k] = (real)((k & 1) ? 1.5 : -1.5);
        centers[3 * k + 1] = (real)((k & 2) ? 1.5 : -1.5);
        centers[3 * k + 2] = (real)-5.0;
        offsets[k] = (real)3.0;
    }
    /* camera at (0.3, -0.2, -6) looking along +z (R = I), OpenCV axes */
    orc_camera cam;
    memset(&cam, 0, sizeof cam);
    cam.width = W;
    cam.height = H;
    cam.fx = cam.fy = (real)(0.5 * W / tan(M_PI / 6.0));
    cam.cx = (real)(0.5 * W);
    cam.cy = (real)(0.5 * H);
    cam.R[0] = cam.R[4] = cam.R[8] = 1;
    cam.pos[0] = (real)0.3; cam.pos[1] = (real)-0.2; cam.pos[2] = (real)-6.0;
    for (int j = 0; j < 3; j++) cam.t[j] = -cam.pos[j];
    cam.znear = (real)0.2;
    cam.lim_x = (real)(1.3 * 0.5 * W / cam.fx);
    cam.lim_y = (real)(1.3 * 0.5 * H / cam.fy);

    int32_t f, o;
    real t;
    if (orc_chunk_pair(centers, K, (real)1.0, cam.pos, &f, &o, &t) != 0) FAIL("chunk_pair");
    real Y[16];
    orc_sh_basis((real)0.6, (real)0.0, (real)0.8, Y);

    const int64_t N = n[0] + n[1];
    uint32_t* ids = must(sizeof(uint32_t) * N);
    real* w = must(sizeof(real) * N);
    for (int mode = 0; mode < 3; mode++) {
        const int64_t c = orc_select(lv, L, d, mode, centers, offsets, K, (real)1.0, cam.pos, ids, w, N, &f, &o, &t);
        if (c < 0 || c > N) FAIL("select mode %d", mode);
    }
    for (int k = 0; k < K; k++)
        if (orc_select_chunk(lv, L, d, centers, offsets, K, k, ids, w, N) < 0) FAIL("select_chunk %d", k);
    const int64_t count = orc_select(lv, L, d, 2, centers, offsets, K, (real)1.0, cam.pos, ids, w, N, &f, &o, &t);

    real* depth = must(sizeof(real) * count);
    real* uv = must(sizeof(real) * 2 * count);
    real* conic = must(sizeof(real) * 3 * count);
    real* o_eff = must(sizeof(real) * count);
    real* rgb = must(sizeof(real) * 3 * count);
    int32_t* rect = must(sizeof(int32_t) * 4 * count);
    uint32_t* tiles = must(sizeof(uint32_t) * count);
    real* radius = must(sizeof(real) * count);
    orc_project(lv, L, ids, w, count, &cam, (real)0.3, 1, depth, uv, conic, o_eff, rgb, rect, tiles, radius);

    const int32_t TX = (W + TILE - 1) / TILE, TY = (H + TILE - 1) / TILE;
    int64_t M = 0;
    for (int64_t a = 0; a < count; a++) M += tiles[a];
    uint32_t* otile = must(sizeof(uint32_t) * M);
    uint64_t* dkey = must(sizeof(uint64_t) * M);
    uint32_t* vals = must(sizeof(uint32_t) * M);
    uint32_t* ranges = must(sizeof(uint32_t) * 2 * TX * TY);
    if (orc_bin_sort(count, depth, rect, tiles, TX, TY, otile, dkey, vals, M, ranges) != M) FAIL("bin_sort");

    real* img = must(sizeof(real) * 3 * W * H);
    real* T = must(sizeof(real) * W * H);
    uint32_t* nc = must(sizeof(uint32_t) * W * H);
    uint32_t* nb = must(sizeof(uint32_t) * W * H);
    uint32_t* ne = must(sizeof(uint32_t) * W * H);
    uint8_t* near = must((size_t)W * H);
    orc_composite(&cam, uv, conic, o_eff, rgb, ranges, vals, img, T, nc, nb, ne, near);
    real* img_b = must(sizeof(real) * 3 * W * H);
    real* T_b = must(sizeof(real) * W * H);
    uint32_t* nc_b = must(sizeof(uint32_t) * W * H);
    orc_composite_brute(&cam, count, depth, rect, tiles, uv, conic, o_eff, rgb, img_b, T_b, nc_b);
    if (memcmp(img, img_b, sizeof(real) * 3 * W * H) || memcmp(T, T_b, sizeof(real) * W * H))
        FAIL("tiled and brute-force compositing differ");

    int32_t xs[3] = {0, W / 2, W - 1}, ys[3] = {0, H / 2, H - 1};
    real col[9], Tp[3];
    uint32_t ncp[3];
    uint8_t nearp[3];
    orc_composite_pixels(&cam, uv, conic, o_eff, rgb, ranges, vals, 3, xs, ys, col, Tp, ncp, nearp);
    const int64_t pm = (int64_t)(H / 2) * W + W / 2;
    const real probe[3] = {img[pm], img[(int64_t)W * H + pm], img[2 * (int64_t)W * H + pm]};
    if (!orc_pixel_accept(&cam, uv, conic, o_eff, rgb, ranges, vals, W / 2, H / 2, probe, (real)1e-4))
        FAIL("pixel_accept rejects the compositor's own value");

    real* score = must(sizeof(real) * N);
    uint8_t* amb = must((size_t)N);
    orc_importance(&cam, uv, conic, o_eff, rgb, ranges, vals, ids, score, amb);
    const int64_t cap = M > 0 ? M : 1;
    uint32_t* act = must(sizeof(uint32_t) * cap);
    real* wt = must(sizeof(real) * cap);
    int64_t* pos = must(sizeof(int64_t) * cap);
    int64_t near_pos = 0;
    if (orc_pixel_weights(&cam, uv, conic, o_eff, rgb, ranges, vals, W / 2, H / 2, act, wt, pos, cap, &near_pos) < 0)
        FAIL("pixel_weights");

    real* dL = must(sizeof(real) * 3 * W * H);
    for (int64_t i = 0; i < 3 * (int64_t)W * H; i++) dL[i] = (real)(uni() - 0.5);
    real* g2 = must(sizeof(real) * 9 * count);
    orc_composite_grad2d(&cam, uv, conic, o_eff, rgb, ranges, vals, dL, g2);
    orc_grads grads[L];
    for (int l = 0; l < L; l++) {
        grads[l].mean = must(sizeof(real) * 3 * n[l]);
        grads[l].scale = must(sizeof(real) * 3 * n[l]);
        grads[l].quat = must(sizeof(real) * 4 * n[l]);
        grads[l].opacity = must(sizeof(real) * n[l]);
        grads[l].sh = must(sizeof(real) * 48 * n[l]);
    }
    orc_project_grad(lv, L, ids, w, count, &cam, (real)0.3, 1, g2, -1, grads);
    orc_project_grad(lv, L, ids, w, count, &cam, (real)0.3, 1, g2, 1, grads);

    printf("ok: %lld selected, %lld instances\n", (long long)count, (long long)M);
    for (int l = 0; l < L; l++) {
        for (int p = 0; p < 5; p++) free(planes[l][p]);
        free(grads[l].mean); free(grads[l].scale); free(grads[l].quat); free(grads[l].opacity); free(grads[l].sh);
    }
    free(ids); free(w); free(depth); free(uv); free(conic); free(o_eff); free(rgb); free(rect); free(tiles);
    free(radius); free(otile); free(dkey); free(vals); free(ranges); free(img); free(T); free(nc); free(nb);
    free(ne); free(near); free(img_b); free(T_b); free(nc_b); free(score); free(amb); free(act); free(wt); free(pos);
    free(dL); free(g2);
    return 0;
}
