/*
 * oracle_sanitize.c -- drives every entry point of the CPU oracle on small
 * ragged inputs, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitize.py).  Test infrastructure: it links
 * oracle/oracle.c only.  Inputs are made here with a fixed linear
 * congruential generator (nothing of the method's arithmetic).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t ortho;
    float eye[3], dir00[3], du[3], dv[3];
} orc_camera;

int orc_brick_minmax(const void *, int, int, int, int, int, double *, double *);
int orc_tf_prefix(const float *, int, int32_t *);
int64_t orc_classify(const double *, const double *, int64_t, int, float, float, const float *, int, uint8_t *);
int64_t orc_vote(const void *, int, int, int, int, int, float, float, const float *, int, uint8_t *);
int64_t orc_tight_boxes(const void *, int, int, int, int, float, float, const float *, int, int, const uint8_t *,
                        int32_t *);
int64_t orc_compact(const uint8_t *, int64_t, uint32_t *);
uint32_t orc_morton3(uint32_t, uint32_t, uint32_t);
int orc_morton_keys(const uint32_t *, int64_t, int, int, uint32_t *);
int orc_sort_pairs(uint32_t *, uint32_t *, int64_t);
int orc_lbvh(const uint32_t *, const uint32_t *, int64_t, int, int, int, int, int, int, uint32_t *, uint32_t *,
             int32_t *, int32_t *, int32_t *);
int64_t orc_kd(const uint8_t *, int, int, int, int, int, int, int, int, int, int, int64_t, int32_t *, int32_t *,
               int32_t *, int32_t *, int32_t *, int32_t *, const int32_t *);
int orc_render(const void *, int, int, int, int, float, float, const float *, int, const orc_camera *, int, int,
               float, float, int, const uint8_t *, int, const int32_t *, int64_t, double *, int64_t *,
               const int32_t *);
int orc_ray(const orc_camera *, int, int, float *, float *);
int orc_sample(const void *, int, int, int, int, float, float, const float *, int, const float *, int64_t,
               double *);

static uint32_t lcg_state = 12345u;
static uint32_t lcg(void)
{
    lcg_state = lcg_state * 1664525u + 1013904223u;
    return lcg_state >> 8;
}

static int check(int ok, const char *what)
{
    if (!ok) fprintf(stderr, "failed: %s\n", what);
    return ok ? 0 : 1;
}

/* one pass of every function over one volume of `dtype` (0 u8, 1 u16, 2 f16, 3 f32) */
static int run(int dtype, int nx, int ny, int nz, int B, int N)
{
    const size_t nvox = (size_t)nx * ny * nz;
    const size_t esz = dtype == 0 ? 1 : (dtype == 3 ? 4 : 2);
    unsigned char *vol = malloc(nvox * esz);
    int bad = 0;
    for (size_t i = 0; i < nvox; ++i) {
        const uint32_t r = lcg();
        const int on = (r % 100) < 20;
        if (dtype == 0) vol[i] = on ? (unsigned char)(r >> 8) : 0;
        else if (dtype == 1) ((uint16_t *)vol)[i] = on ? (uint16_t)(r >> 4) : 0;
        else if (dtype == 2) ((uint16_t *)vol)[i] = on ? (uint16_t)(0x3000 + (r % 0xC00)) : 0; /* [0.125, 1) */
        else ((float *)vol)[i] = on ? (float)(r % 1000) / 999.0f : 0.0f;
    }
    float *tf = malloc(sizeof(float) * 4 * (size_t)N);
    for (int i = 0; i < N; ++i) {
        tf[4 * i + 0] = (float)i / (float)(N - 1);
        tf[4 * i + 1] = 0.5f;
        tf[4 * i + 2] = 1.0f - (float)i / (float)(N - 1);
        tf[4 * i + 3] = i < N / 3 ? 0.0f : 0.6f * (float)(i - N / 3) / (float)N;
    }
    tf[4 * (N - 1) + 3] = NAN; /* read as 0 */
    tf[4 * (N / 2) + 3] = 3.0f; /* read as 1 */
    const int nbx = (nx + B - 1) / B, nby = (ny + B - 1) / B, nbz = (nz + B - 1) / B;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    double *mn = malloc(sizeof(double) * nb), *mx = malloc(sizeof(double) * nb);
    bad += check(orc_brick_minmax(vol, dtype, nx, ny, nz, B, mn, mx) == 0, "minmax");
    int32_t *P = malloc(sizeof(int32_t) * (N + 1));
    bad += check(orc_tf_prefix(tf, N, P) == 0, "prefix");
    uint8_t *flags = malloc(nb), *vflags = malloc(nb);
    const int64_t n = orc_classify(mn, mx, nb, dtype, -0.25f, 1.25f, tf, N, flags);
    bad += check(n >= 0 && n <= nb, "classify");
    bad += check(orc_vote(vol, dtype, nx, ny, nz, B, -0.25f, 1.25f, tf, N, vflags) >= 0, "vote");
    int32_t *boxes = malloc(sizeof(int32_t) * 6 * nb);
    bad += check(orc_tight_boxes(vol, dtype, nx, ny, nz, -0.25f, 1.25f, tf, N, B, flags, boxes) >= 0, "tight");
    uint32_t *ids = malloc(sizeof(uint32_t) * (nb + 1)), *keys = malloc(sizeof(uint32_t) * (nb + 1));
    bad += check(orc_compact(flags, nb, ids) == n, "compact");
    orc_morton_keys(ids, n, nbx, nby, keys);
    bad += check(orc_sort_pairs(keys, ids, n) == 0, "sort");
    const int64_t m = n > 1 ? n - 1 : 1;
    uint32_t *left = malloc(sizeof(uint32_t) * m), *right = malloc(sizeof(uint32_t) * m);
    int32_t *axis = malloc(sizeof(int32_t) * m), *lo = malloc(sizeof(int32_t) * 3 * m),
            *hi = malloc(sizeof(int32_t) * 3 * m);
    bad += check(orc_lbvh(keys, ids, n, nbx, nby, B, nx, ny, nz, left, right, axis, lo, hi) >= 0, "lbvh");
    const int64_t cap = 2 * nb;
    int32_t *klo = malloc(sizeof(int32_t) * 3 * cap), *khi = malloc(sizeof(int32_t) * 3 * cap);
    int32_t *kax = malloc(sizeof(int32_t) * cap), *kpl = malloc(sizeof(int32_t) * cap),
            *kfc = malloc(sizeof(int32_t) * cap), height = 0;
    const int variants[6][3] = {{0, 0, 4}, {1, 0, 4}, {1, 16, 4}, {1, 0, 2}, {0, 0, 3}, {1, 8, 16}};
    for (int v = 0; v < 12; ++v)
        bad += check(orc_kd(flags, nbx, nby, nbz, B, nx, ny, nz, variants[v % 6][0], variants[v % 6][1],
                            variants[v % 6][2], cap, klo, khi, kax, kpl, kfc, &height, v < 6 ? NULL : boxes) >= 0,
                     "kd");
    orc_camera cam = {0, {-30.0f, (float)ny * 0.5f, -40.0f}, {0.6f, -0.05f, 0.8f}, {0.01f, 0.0f, -0.008f},
                      {0.0f, -0.012f, 0.0f}};
    const int W = 21, H = 17;
    double *img = malloc(sizeof(double) * 4 * W * H);
    int64_t *cnt = malloc(sizeof(int64_t) * W * H);
    for (int mode = 0; mode < 3; ++mode)
        bad += check(orc_render(vol, dtype, nx, ny, nz, -0.25f, 1.25f, tf, N, &cam, W, H, 0.5f, 1.0f, mode, flags, B,
                                NULL, 0, img, cnt, boxes) == 0,
                     "render");
    cam.ortho = 1;
    const int32_t pix[6] = {0, 0, W - 1, H - 1, 10, 8};
    bad += check(orc_render(vol, dtype, nx, ny, nz, -0.25f, 1.25f, tf, N, &cam, W, H, 0.37f, 0.0f, 0, NULL, 0, pix,
                            3, img, cnt, NULL) == 0,
                 "render pixels");
    float o[3], d[3], pts[6] = {0.1f, 0.2f, 0.3f, (float)nx - 0.01f, (float)ny - 0.01f, (float)nz - 0.01f};
    double rgba[8];
    orc_ray(&cam, 3, 4, o, d);
    bad += check(orc_sample(vol, dtype, nx, ny, nz, -0.25f, 1.25f, tf, N, pts, 2, rgba) == 0, "sample");
    bad += check(orc_morton3(1023, 1023, 1023) == (1u << 30) - 1u, "morton");
    free(vol); free(tf); free(mn); free(mx); free(P); free(flags); free(vflags); free(boxes); free(ids); free(keys);
    free(left); free(right); free(axis); free(lo); free(hi); free(klo); free(khi); free(kax); free(kpl); free(kfc);
    free(img); free(cnt);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad += run(0, 37, 29, 23, 8, 256);
    bad += run(1, 19, 33, 17, 4, 300);
    bad += run(2, 25, 18, 31, 8, 64);
    bad += run(3, 33, 20, 26, 16, 1024);
    bad += run(0, 1, 1, 1, 4, 2);     /* a single voxel, two TF entries */
    if (bad) return 1;
    printf("oracle sanitizer run ok\n");
    return 0;
}
