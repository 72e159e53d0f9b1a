/*
 * oracle.c -- plain, slow, obviously correct CPU oracle for the empty-space-
 * skipping hot path of "Comparing Hierarchical Data Structures for Sparse
 * Volume Rendering with Empty Space Skipping" (Zellmann et al., arXiv
 * 1912.09596).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product path (the HIP
 * library and its Python binding) never includes, links, imports or calls it,
 * and this file includes nothing from the product.
 *
 * Precision: voxel values, transfer-function lookups and compositing are FP64.
 * Ray geometry (ray origin/direction, slab entry/exit, the sample positions
 * p_k and their membership tests) is FP32 on purpose: the sample set of a
 * discretised ray is a discrete object, and both implementations must agree
 * on it exactly, so both evaluate the same FP32 formulas without contraction
 * (build with -ffp-contract=off, no -ffast-math).  Classification indices of
 * float volumes are likewise taken in FP32 (the precision the device decides
 * them in); for integer volumes they are exact integers.
 *
 * Layout conventions (shared by contract with the device library, not by
 * code): voxel (x,y,z) lives at x + nx*(y + ny*z); brick b = (bx,by,bz) of edge
 * B covers voxels [B*b, min(B*b+B, n)) per axis; linear brick id
 * bx + nbx*(by + nby*bz); transfer functions are N x RGBA float32.
 *
 * Parity pins for every function below live in tests/test_oracle_*.py.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_U8 = 0, ORC_U16 = 1, ORC_F16 = 2, ORC_F32 = 3 };

/* ------------------------------------------------------------------------ */
/* voxel access                                                              */
/* ------------------------------------------------------------------------ */

/* IEEE binary16 -> double, written out from the format definition. */
static double half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int expo = (h >> 10) & 0x1f;
    int mant = h & 0x3ff;
    double v;
    if (expo == 0)
        v = ldexp((double)mant, -24); /* subnormal: mant * 2^-14 * 2^-10 */
    else if (expo == 31)
        v = mant ? NAN : INFINITY;
    else
        v = ldexp((double)(mant | 0x400), expo - 25);
    return sign ? -v : v;
}

static double voxel(const void *vol, int dtype, size_t i)
{
    switch (dtype) {
    case ORC_U8: return (double)((const uint8_t *)vol)[i];
    case ORC_U16: return (double)((const uint16_t *)vol)[i];
    case ORC_F16: return half_to_double(((const uint16_t *)vol)[i]);
    default: return (double)((const float *)vol)[i];
    }
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/* ------------------------------------------------------------------------ */
/* a1: per-brick min/max with a one-voxel apron.                             */
/* Sec. 3.1 decomposes the volume into bricks and decides per brick whether  */
/* anything in it is visible; Sec. 2 names min-max range queries as the way  */
/* to classify a region without touching its voxels.  The apron is the       */
/* trilinear footprint of the samples a brick owns.                          */
/* ------------------------------------------------------------------------ */
int orc_brick_minmax(const void *vol, int dtype, int nx, int ny, int nz, int B,
                     double *mn, double *mx)
{
    if (!vol || nx < 1 || ny < 1 || nz < 1 || B < 1) return -1;
    int nbx = (int)ceil_div(nx, B), nby = (int)ceil_div(ny, B), nbz = (int)ceil_div(nz, B);
    for (int bz = 0; bz < nbz; ++bz)
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                int x0 = clampi(B * bx - 1, 0, nx - 1), x1 = clampi(B * bx + B, 0, nx - 1);
                int y0 = clampi(B * by - 1, 0, ny - 1), y1 = clampi(B * by + B, 0, ny - 1);
                int z0 = clampi(B * bz - 1, 0, nz - 1), z1 = clampi(B * bz + B, 0, nz - 1);
                double lo = INFINITY, hi = -INFINITY;
                for (int z = z0; z <= z1; ++z)
                    for (int y = y0; y <= y1; ++y)
                        for (int x = x0; x <= x1; ++x) {
                            double v = voxel(vol, dtype, (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z));
                            if (v < lo) lo = v;
                            if (v > hi) hi = v;
                        }
                size_t b = (size_t)bx + (size_t)nbx * ((size_t)by + (size_t)nby * bz);
                mn[b] = lo;
                mx[b] = hi;
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Opacity of TF entry i as every step below reads it: the paper leaves the  */
/* TF's value range unstated; an opacity is a fraction, so values above 1    */
/* count as 1 and negative or NaN values as 0 (fully transparent).  Colour   */
/* is used as given.                                                          */
/* ------------------------------------------------------------------------ */
static float tf_alpha(const float *tf, int i)
{
    float a = tf[4 * i + 3];
    if (!(a > 0.0f)) return 0.0f; /* also NaN */
    return a > 1.0f ? 1.0f : a;
}

/* ------------------------------------------------------------------------ */
/* a2: prefix count of visible transfer-function entries,                    */
/* P[0] = 0, P[i+1] = P[i] + (alpha_i > 0).  (The range-query table the      */
/* commented-out note under the statistics table prices at 1024 entries.)    */
/* ------------------------------------------------------------------------ */
int orc_tf_prefix(const float *tf, int N, int32_t *P)
{
    if (!tf || N < 2) return -1;
    P[0] = 0;
    for (int i = 0; i < N; ++i) P[i + 1] = P[i] + (tf_alpha(tf, i) > 0.0f ? 1 : 0);
    return 0;
}

/* floor of the transfer-function coordinate x(v) = s(v) * (N-1). */
static int64_t tf_floor_index(double v, int dtype, float lo, float hi, int N)
{
    if (dtype == ORC_U8) return ((int64_t)v * (N - 1)) / 255;
    if (dtype == ORC_U16) return ((int64_t)v * (N - 1)) / 65535;
    {
        float fv = (float)v;
        float num = fv - lo;
        float den = hi - lo;
        float s = num / den;
        if (s < 0.0f) s = 0.0f;
        if (s > 1.0f) s = 1.0f;
        float x = s * (float)(N - 1);
        return (int64_t)floorf(x);
    }
}

/* ------------------------------------------------------------------------ */
/* a3: brick classification.  A brick is non-empty iff some entry in         */
/* [floor(x(min))-1, floor(x(max))+2] clamped to [0,N-1] has alpha > 0.      */
/* Sec. 3.1: bricks are classified visible/invisible under the current       */
/* transfer function whenever it changes.  The window is every entry a       */
/* sample owned by the brick can read with a non-zero lerp weight: a value   */
/* in [min, max] reads entries floor(x) and ceil(x) <= floor(x(max)) + 1,   */
/* and one more entry on each side absorbs rounding of the interpolated     */
/* value (ceil of a value rounded just past an integer).                     */
/* ------------------------------------------------------------------------ */
int64_t orc_classify(const double *mn, const double *mx, int64_t nb, int dtype, float lo,
                     float hi, const float *tf, int N, uint8_t *flags)
{
    if (!mn || !mx || !tf || !flags || N < 2) return -1;
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    if (!P) return -1;
    orc_tf_prefix(tf, N, P);
    int64_t count = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t a = tf_floor_index(mn[b], dtype, lo, hi, N) - 1;
        int64_t c = tf_floor_index(mx[b], dtype, lo, hi, N) + 2;
        if (a < 0) a = 0;
        if (c > N - 1) c = N - 1;
        flags[b] = (P[c + 1] - P[a]) > 0 ? 1 : 0;
        count += flags[b];
    }
    free(P);
    return count;
}

/* ------------------------------------------------------------------------ */
/* a3 variant: the per-voxel vote of Sec. 3.1.  A brick is non-empty iff one */
/* of its own voxels (no apron) is visible: alpha > 0 under the renderer's   */
/* TF lookup.  The lookup decides an integer flag, so it is taken in the     */
/* device's precision, FP32: s = (v - lo) * scale with scale = 1/255 (u8),   */
/* 1/65535 (u16) or 1/(hi - lo) (f16, f32), x = clamp(s, 0, 1) * (N - 1),    */
/* i0 = min(trunc(x), N - 2), alpha = fmaf(x - i0, a[i0+1] - a[i0], a[i0]).  */
/* ------------------------------------------------------------------------ */
int64_t orc_vote(const void *vol, int dtype, int nx, int ny, int nz, int B, float lo, float hi,
                 const float *tf, int N, uint8_t *flags)
{
    if (!vol || !tf || !flags || N < 2 || B < 1) return -1;
    float nlo = 0.0f, nscale;
    if (dtype == ORC_U8)
        nscale = 1.0f / 255.0f;
    else if (dtype == ORC_U16)
        nscale = 1.0f / 65535.0f;
    else {
        nlo = lo;
        nscale = 1.0f / (hi - lo);
    }
    const int64_t nbx = ceil_div(nx, B), nby = ceil_div(ny, B), nbz = ceil_div(nz, B);
    memset(flags, 0, (size_t)(nbx * nby * nbz));
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t b = x / B + nbx * (y / B + nby * (int64_t)(z / B));
                if (flags[b]) continue;
                const float v = (float)voxel(vol, dtype, (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z));
                float t = (v - nlo) * nscale;
                t = t < 0.0f ? 0.0f : (t > 1.0f ? 1.0f : t);
                t = t * (float)(N - 1);
                int i0 = (int)t;
                if (i0 > N - 2) i0 = N - 2;
                const float f = t - (float)i0;
                const float a0 = tf_alpha(tf, i0), a1 = tf_alpha(tf, i0 + 1);
                if (fmaf(f, a1 - a0, a0) > 0.0f) flags[b] = 1;
            }
    int64_t count = 0;
    for (int64_t b = 0; b < nbx * nby * nbz; ++b) count += flags[b];
    return count;
}

/* ------------------------------------------------------------------------ */
/* Voxel-tight brick boxes (the GPU k-d variant of Sec. 3.2.2 keeps a tight  */
/* box per macro cell, recomputed when the TF changes).  A sample point p    */
/* reads the trilinear cell c = floor(p - 1/2) per axis (its 8 corner voxels */
/* clamped to the volume), whose region is [c + 1/2, c + 3/2).  A cell is    */
/* potentially visible iff the classification window of its 8 values holds  */
/* an entry with alpha > 0 (the brick test above, on the cell's own min/max).*/
/* A brick's tight box is the bounding box of the regions of its potentially */
/* visible cells, clipped to the brick, in half-voxel units (lo2, hi2 per    */
/* axis, the box being [lo2/2, hi2/2)).  Samples outside it read only        */
/* invisible cells: alpha exactly 0.  Unflagged bricks and bricks without a  */
/* visible cell get the empty box (all zero).                                */
/* ------------------------------------------------------------------------ */
int64_t orc_tight_boxes(const void *vol, int dtype, int nx, int ny, int nz, float lo, float hi, const float *tf,
                        int N, int B, const uint8_t *flags, int32_t *boxes)
{
    if (!vol || !tf || !flags || !boxes || N < 2 || B < 1) return -1;
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    if (!P) return -1;
    orc_tf_prefix(tf, N, P);
    const int n[3] = {nx, ny, nz};
    const int64_t nb[3] = {ceil_div(nx, B), ceil_div(ny, B), ceil_div(nz, B)};
    const int64_t total = nb[0] * nb[1] * nb[2];
    int64_t nonempty = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nonempty)
    for (int64_t b = 0; b < total; ++b) {
        int32_t *box = boxes + 6 * b;
        for (int a = 0; a < 6; ++a) box[a] = 0;
        if (!flags[b]) continue;
        const int bc[3] = {(int)(b % nb[0]), (int)((b / nb[0]) % nb[1]), (int)(b / (nb[0] * nb[1]))};
        int blo[3], bhi[3], tlo[3], thi[3];
        for (int a = 0; a < 3; ++a) {
            blo[a] = bc[a] * B;
            bhi[a] = blo[a] + B < n[a] ? blo[a] + B : n[a];
            tlo[a] = 2 * bhi[a];
            thi[a] = 2 * blo[a];
        }
        int any = 0;
        /* cells whose region [c + 1/2, c + 3/2) meets the brick [blo, bhi) */
        for (int cz = blo[2] - 1; cz <= bhi[2] - 1; ++cz)
            for (int cy = blo[1] - 1; cy <= bhi[1] - 1; ++cy)
                for (int cx = blo[0] - 1; cx <= bhi[0] - 1; ++cx) {
                    const int c[3] = {cx, cy, cz};
                    double mn = INFINITY, mx = -INFINITY;
                    for (int corner = 0; corner < 8; ++corner) {
                        int q[3];
                        for (int a = 0; a < 3; ++a) q[a] = clampi(c[a] + ((corner >> a) & 1), 0, n[a] - 1);
                        const double v =
                            voxel(vol, dtype, (size_t)q[0] + (size_t)nx * ((size_t)q[1] + (size_t)ny * q[2]));
                        if (v < mn) mn = v;
                        if (v > mx) mx = v;
                    }
                    int64_t wlo = tf_floor_index(mn, dtype, lo, hi, N) - 1;
                    int64_t whi = tf_floor_index(mx, dtype, lo, hi, N) + 2;
                    if (wlo < 0) wlo = 0;
                    if (whi > N - 1) whi = N - 1;
                    if (P[whi + 1] - P[wlo] <= 0) continue;
                    any = 1;
                    for (int a = 0; a < 3; ++a) {
                        const int l2 = 2 * c[a] + 1 > 2 * blo[a] ? 2 * c[a] + 1 : 2 * blo[a];
                        const int h2 = 2 * c[a] + 3 < 2 * bhi[a] ? 2 * c[a] + 3 : 2 * bhi[a];
                        if (l2 < tlo[a]) tlo[a] = l2;
                        if (h2 > thi[a]) thi[a] = h2;
                    }
                }
        if (!any) continue;
        for (int a = 0; a < 3; ++a) {
            box[a] = tlo[a];
            box[3 + a] = thi[a];
        }
        nonempty += 1;
    }
    free(P);
    return nonempty;
}

/* a4: compaction -- ids of the non-empty bricks in ascending linear id (Sec. 3.1). */
int64_t orc_compact(const uint8_t *flags, int64_t nb, uint32_t *ids)
{
    int64_t n = 0;
    for (int64_t b = 0; b < nb; ++b)
        if (flags[b]) ids[n++] = (uint32_t)b;
    return n;
}

/* a5: 30-bit 3-D Morton code, 10 bits per axis; bit i of x goes to bit 3i+2,
 * of y to 3i+1, of z to 3i (Sec. 3.1). */
uint32_t orc_morton3(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t code = 0;
    for (int i = 0; i < 10; ++i) {
        code |= ((x >> i) & 1u) << (3 * i + 2);
        code |= ((y >> i) & 1u) << (3 * i + 1);
        code |= ((z >> i) & 1u) << (3 * i);
    }
    return code;
}

int orc_morton_keys(const uint32_t *ids, int64_t n, int nbx, int nby, uint32_t *keys)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t id = ids[i];
        uint32_t x = id % (uint32_t)nbx;
        uint32_t y = (id / (uint32_t)nbx) % (uint32_t)nby;
        uint32_t z = id / ((uint32_t)nbx * (uint32_t)nby);
        keys[i] = orc_morton3(x, y, z);
    }
    return 0;
}

/* a6: sort (key, id) pairs by key.  Keys of distinct bricks are distinct, so
 * the order is unique.  The library sort is the step (Sec. 3.1 uses a
 * radix sort; any correct sort gives the same unique order). */
typedef struct { uint32_t key, id; } orc_pair;
static int cmp_pair(const void *a, const void *b)
{
    uint32_t ka = ((const orc_pair *)a)->key, kb = ((const orc_pair *)b)->key;
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}
int orc_sort_pairs(uint32_t *keys, uint32_t *ids, int64_t n)
{
    orc_pair *p = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
    if (!p) return -1;
    for (int64_t i = 0; i < n; ++i) { p[i].key = keys[i]; p[i].id = ids[i]; }
    qsort(p, (size_t)n, sizeof(orc_pair), cmp_pair);
    for (int64_t i = 0; i < n; ++i) { keys[i] = p[i].key; ids[i] = p[i].id; }
    free(p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* a7 + a8: the radix tree over sorted Morton codes, numbered as in Karras's */
/* scheme (root = internal node 0; a range [f,l] split after index s has its */
/* left child at s and its right child at s+1, each a leaf when its range is */
/* a single key), and the bottom-up AABB union (Sec. 3.1).  Written as the   */
/* plain top-down recursion over ranges: the split of [f,l] is the last      */
/* index whose key still has a 0 at the highest bit where key[f] and key[l]  */
/* differ.                                                                    */
/* ------------------------------------------------------------------------ */
#define ORC_LEAF 0x80000000u

typedef struct {
    const uint32_t *keys, *ids;
    int nbx, nby, B, n[3];
    uint32_t *left, *right;
    int32_t *axis, *lo, *hi; /* lo/hi: [N-1][3] internal boxes in voxels */
} lbvh_ctx;

static void brick_box(const lbvh_ctx *c, uint32_t id, int lo[3], int hi[3])
{
    int b[3];
    b[0] = (int)(id % (uint32_t)c->nbx);
    b[1] = (int)((id / (uint32_t)c->nbx) % (uint32_t)c->nby);
    b[2] = (int)(id / ((uint32_t)c->nbx * (uint32_t)c->nby));
    for (int a = 0; a < 3; ++a) {
        lo[a] = c->B * b[a];
        hi[a] = c->B * b[a] + c->B;
        if (hi[a] > c->n[a]) hi[a] = c->n[a];
    }
}

/* builds the subtree over [f,l] whose node index is `node`; returns height */
static int lbvh_rec(lbvh_ctx *c, int64_t f, int64_t l, int64_t node, int lo[3], int hi[3])
{
    uint32_t diff = c->keys[f] ^ c->keys[l];
    int bit = 31;
    while (!((diff >> bit) & 1u)) --bit; /* keys are distinct, so diff != 0 */
    int64_t s = f;
    while (s + 1 <= l && !((c->keys[s + 1] >> bit) & 1u)) ++s; /* last 0 at `bit` */
    c->axis[node] = 2 - (bit % 3);
    int llo[3], lhi[3], rlo[3], rhi[3], hl, hr;
    if (s == f) {
        c->left[node] = ORC_LEAF | (uint32_t)s;
        brick_box(c, c->ids[s], llo, lhi);
        hl = 1;
    } else {
        c->left[node] = (uint32_t)s;
        hl = lbvh_rec(c, f, s, s, llo, lhi);
    }
    if (s + 1 == l) {
        c->right[node] = ORC_LEAF | (uint32_t)(s + 1);
        brick_box(c, c->ids[s + 1], rlo, rhi);
        hr = 1;
    } else {
        c->right[node] = (uint32_t)(s + 1);
        hr = lbvh_rec(c, s + 1, l, s + 1, rlo, rhi);
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] = llo[a] < rlo[a] ? llo[a] : rlo[a];
        hi[a] = lhi[a] > rhi[a] ? lhi[a] : rhi[a];
        c->lo[3 * node + a] = lo[a];
        c->hi[3 * node + a] = hi[a];
    }
    return 1 + (hl > hr ? hl : hr);
}

/* Returns the tree height in levels (1 for a single leaf, 0 for no bricks). */
int orc_lbvh(const uint32_t *sorted_keys, const uint32_t *sorted_ids, int64_t n, int nbx, int nby,
             int B, int nx, int ny, int nz, uint32_t *left, uint32_t *right, int32_t *axis,
             int32_t *lo, int32_t *hi)
{
    if (n <= 0) return 0;
    if (n == 1) return 1;
    lbvh_ctx c = {sorted_keys, sorted_ids, nbx, nby, B, {nx, ny, nz}, left, right, axis, lo, hi};
    int rlo[3], rhi[3];
    return lbvh_rec(&c, 0, n - 1, 0, rlo, rhi);
}

/* ------------------------------------------------------------------------ */
/* a10: binned k-d tree over the brick occupancy (Sec. 3.2, 3.2.2, 4.3).     */
/* Top-down, breadth first.  Each node keeps the tight box (in bricks) of    */
/* the non-empty bricks inside its region.  Candidate planes lie on bin      */
/* boundaries of the brick raster (4 bins -> planes at lo + floor(j*e/4)).   */
/* Cost of a plane = voxel volume of the tight box left of it plus that of   */
/* the tight box right of it; split iff the best cost is strictly below the  */
/* node's volume.  Halting: shallow = split only while 10*V > V(root); deep */
/* = split only while V > 8^3.  Maximum leaf size: when the cost says leaf   */
/* and V > MLS^3, split in the middle of the axis with the largest extent.   */
/* Tight boxes are found here by scanning the flags (the plain definition).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *flags;
    int nb[3], B, n[3];
} kd_ctx;

static int kd_flag(const kd_ctx *c, int x, int y, int z)
{
    return c->flags[(size_t)x + (size_t)c->nb[0] * ((size_t)y + (size_t)c->nb[1] * z)] != 0;
}

/* tight box of the non-empty bricks in region [rlo, rhi); returns 0 if none */
static int kd_tight(const kd_ctx *c, const int rlo[3], const int rhi[3], int tlo[3], int thi[3])
{
    int found = 0;
    for (int z = rlo[2]; z < rhi[2]; ++z)
        for (int y = rlo[1]; y < rhi[1]; ++y)
            for (int x = rlo[0]; x < rhi[0]; ++x)
                if (kd_flag(c, x, y, z)) {
                    int p[3] = {x, y, z};
                    if (!found) {
                        for (int a = 0; a < 3; ++a) { tlo[a] = p[a]; thi[a] = p[a] + 1; }
                        found = 1;
                    } else {
                        for (int a = 0; a < 3; ++a) {
                            if (p[a] < tlo[a]) tlo[a] = p[a];
                            if (p[a] + 1 > thi[a]) thi[a] = p[a] + 1;
                        }
                    }
                }
    return found;
}

/* voxel volume of a box given in bricks, clipped to the volume */
static int64_t kd_volume(const kd_ctx *c, const int lo[3], const int hi[3])
{
    int64_t v = 1;
    for (int a = 0; a < 3; ++a) {
        int64_t e1 = (int64_t)c->B * hi[a];
        if (e1 > c->n[a]) e1 = c->n[a];
        v *= e1 - (int64_t)c->B * lo[a];
    }
    return v;
}

/* Voxel-tight cost (the GPU builder of Sec. 3.2.2 keeps one voxel-tight box */
/* per macro cell and, for a region spanning several cells, reduces over     */
/* them): the tight box of a region is the union of the voxel-tight boxes    */
/* (half-voxel units, as orc_tight_boxes gives them) of the bricks inside    */
/* it, and its volume is measured in half-voxel units (eight per voxel).     */
/* Returns that volume, 0 when no brick of the region has a visible cell.   */
static int64_t kd_tight_volume(const kd_ctx *c, const int32_t *tbox, const int rlo[3], const int rhi[3])
{
    int found = 0, ulo[3] = {0, 0, 0}, uhi[3] = {0, 0, 0};
    for (int z = rlo[2]; z < rhi[2]; ++z)
        for (int y = rlo[1]; y < rhi[1]; ++y)
            for (int x = rlo[0]; x < rhi[0]; ++x) {
                const int32_t *b = tbox + 6 * ((size_t)x + (size_t)c->nb[0] * ((size_t)y + (size_t)c->nb[1] * z));
                if (!(b[3] > b[0] && b[4] > b[1] && b[5] > b[2])) continue;   /* no visible cell */
                for (int a = 0; a < 3; ++a) {
                    if (!found || b[a] < ulo[a]) ulo[a] = b[a];
                    if (!found || b[3 + a] > uhi[a]) uhi[a] = b[3 + a];
                }
                found = 1;
            }
    if (!found) return 0;
    return (int64_t)(uhi[0] - ulo[0]) * (uhi[1] - ulo[1]) * (uhi[2] - ulo[2]);
}

/* out arrays sized `cap` nodes: lo/hi [cap][3] (bricks), axis (-1 = leaf),
 * plane (bricks, 0 for leaves), first_child (-1 for leaves).  Returns the
 * node count (0 for an empty occupancy), or -1 if cap is too small; the
 * height in levels goes to *height.  tbox: NULL for the brick-granular cost,
 * else the voxel-tight box of every brick ([nb][6], half-voxel units): every
 * volume the build compares (a side's cost, the node, the root, the 8^3 and
 * maximum-leaf-size limits) is then the half-voxel volume of the union of
 * the voxel-tight boxes inside the region; node regions, candidate planes
 * and children stay on the brick raster. */
int64_t orc_kd(const uint8_t *flags, int nbx, int nby, int nbz, int B, int nx, int ny, int nz,
               int halting, int max_leaf, int bins, int64_t cap, int32_t *lo, int32_t *hi,
               int32_t *axis, int32_t *plane, int32_t *first_child, int32_t *height, const int32_t *tbox)
{
    kd_ctx c = {flags, {nbx, nby, nbz}, B, {nx, ny, nz}};
    /* units of the volumes compared: voxels, or half-voxels (8 per voxel) */
    const int64_t unit = tbox ? 8 : 1;
    int glo[3] = {0, 0, 0}, ghi[3] = {nbx, nby, nbz};
    int rlo[3], rhi[3];
    *height = 0;
    if (!kd_tight(&c, glo, ghi, rlo, rhi)) return 0;
    if (cap < 1) return -1;
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    if (!depth) return -1;
    int64_t count = 1, head = 0;
    for (int a = 0; a < 3; ++a) { lo[a] = rlo[a]; hi[a] = rhi[a]; }
    depth[0] = 1;
    int64_t vroot = tbox ? kd_tight_volume(&c, tbox, rlo, rhi) : kd_volume(&c, rlo, rhi);
    while (head < count) {
        int64_t i = head++;
        int blo[3], bhi[3];
        for (int a = 0; a < 3; ++a) { blo[a] = lo[3 * i + a]; bhi[a] = hi[3 * i + a]; }
        if (depth[i] > *height) *height = depth[i];
        int64_t V = tbox ? kd_tight_volume(&c, tbox, blo, bhi) : kd_volume(&c, blo, bhi);
        int allowed = halting == 0 ? (10 * V > vroot) : (V > 512 * unit);
        int best_axis = -1, best_plane = 0;
        int64_t best_cost = 0;
        if (allowed) {
            for (int a = 0; a < 3; ++a) {
                int e = bhi[a] - blo[a];
                if (e < 2) continue;
                int prev = -1;
                for (int j = 1; j < bins; ++j) {
                    int p = blo[a] + (int)(((int64_t)j * e) / bins);
                    if (p <= blo[a] || p >= bhi[a] || p == prev) continue;
                    prev = p;
                    int llo[3], lhi[3], ulo[3], uhi[3], tl[3], th[3], tu[3], tv[3];
                    for (int q = 0; q < 3; ++q) { llo[q] = ulo[q] = blo[q]; lhi[q] = uhi[q] = bhi[q]; }
                    lhi[a] = p;
                    ulo[a] = p;
                    int64_t cost = 0;
                    if (tbox) {
                        cost = kd_tight_volume(&c, tbox, llo, lhi) + kd_tight_volume(&c, tbox, ulo, uhi);
                    } else {
                        if (kd_tight(&c, llo, lhi, tl, th)) cost += kd_volume(&c, tl, th);
                        if (kd_tight(&c, ulo, uhi, tu, tv)) cost += kd_volume(&c, tu, tv);
                    }
                    if (best_axis < 0 || cost < best_cost) {
                        best_axis = a;
                        best_plane = p;
                        best_cost = cost;
                    }
                }
            }
            if (best_axis >= 0 && !(best_cost < V)) {
                best_axis = -1;
                if (max_leaf > 0 && V > (int64_t)max_leaf * max_leaf * max_leaf * unit) {
                    int64_t best_ext = -1;
                    for (int a = 0; a < 3; ++a) {
                        int e = bhi[a] - blo[a];
                        if (e < 2) continue;
                        int64_t e1 = (int64_t)B * bhi[a];
                        if (e1 > c.n[a]) e1 = c.n[a];
                        int64_t ext = e1 - (int64_t)B * blo[a];
                        if (ext > best_ext) { best_ext = ext; best_axis = a; best_plane = blo[a] + e / 2; }
                    }
                }
            }
        }
        if (best_axis < 0) {
            axis[i] = -1;
            plane[i] = 0;
            first_child[i] = -1;
            continue;
        }
        if (count + 2 > cap) { free(depth); return -1; }
        axis[i] = best_axis;
        plane[i] = best_plane;
        first_child[i] = (int32_t)count;
        for (int side = 0; side < 2; ++side) {
            int slo[3], shi[3], tlo[3], thi[3];
            for (int q = 0; q < 3; ++q) { slo[q] = blo[q]; shi[q] = bhi[q]; }
            if (side == 0) shi[best_axis] = best_plane; else slo[best_axis] = best_plane;
            kd_tight(&c, slo, shi, tlo, thi); /* non-empty: the parent box is tight */
            for (int q = 0; q < 3; ++q) { lo[3 * count + q] = tlo[q]; hi[3 * count + q] = thi[q]; }
            depth[count] = depth[i] + 1;
            ++count;
        }
    }
    free(depth);
    return count;
}

/* ------------------------------------------------------------------------ */
/* a11..a14: the image.  The oracle's image is the unskipped full march     */
/* (the "naive" ray marcher of Sec. 4): absorption plus emission, post-      */
/* classification (interpolate the scalar, then look up the transfer         */
/* function), no gradient shading, no early ray termination (Sec. 4.1).      */
/* mode 0: every sample inside the volume is composited.                     */
/* mode 1: only samples whose brick floor(floor(p)/B) is flagged (the        */
/*         self-check that skipping empty bricks changes nothing).           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t ortho;
    float eye[3], dir00[3], du[3], dv[3];
} orc_camera;

static void ray_for_pixel(const orc_camera *cam, int px, int py, float o[3], float d[3])
{
    float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    float v[3];
    for (int a = 0; a < 3; ++a) {
        if (cam->ortho) {
            float t1 = fx * cam->du[a];
            float t2 = fy * cam->dv[a];
            o[a] = (cam->eye[a] + t1) + t2;
            v[a] = cam->dir00[a];
        } else {
            float t1 = fx * cam->du[a];
            float t2 = fy * cam->dv[a];
            o[a] = cam->eye[a];
            v[a] = (cam->dir00[a] + t1) + t2;
        }
    }
    float l2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    float len = sqrtf(l2);
    for (int a = 0; a < 3; ++a) d[a] = v[a] / len;
}

/* ray/box slab test in FP32; 0 if the ray misses the box's slabs */
static int slab(const float o[3], const float d[3], const float lo[3], const float hi[3],
                float *tn, float *tf)
{
    float t0 = -FLT_MAX, t1 = FLT_MAX;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0f) {
            float ta = (lo[a] - o[a]) / d[a];
            float tb = (hi[a] - o[a]) / d[a];
            float mn = ta < tb ? ta : tb;
            float mx = ta < tb ? tb : ta;
            if (mn > t0) t0 = mn;
            if (mx < t1) t1 = mx;
        } else if (o[a] < lo[a] || o[a] >= hi[a]) {
            return 0;
        }
    }
    *tn = t0;
    *tf = t1;
    return 1;
}

/* cell-centred trilinear interpolation (clamp to edge), FP64 */
static double trilinear(const void *vol, int dtype, const int n[3], const float p[3])
{
    int i0[3], i1[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        double u = (double)p[a] - 0.5;
        double fl = floor(u);
        w[a] = u - fl;
        int i = (int)fl;
        i0[a] = clampi(i, 0, n[a] - 1);
        i1[a] = clampi(i + 1, 0, n[a] - 1);
    }
#define V(X, Y, Z) voxel(vol, dtype, (size_t)(X) + (size_t)n[0] * ((size_t)(Y) + (size_t)n[1] * (size_t)(Z)))
    double c00 = V(i0[0], i0[1], i0[2]) + w[0] * (V(i1[0], i0[1], i0[2]) - V(i0[0], i0[1], i0[2]));
    double c10 = V(i0[0], i1[1], i0[2]) + w[0] * (V(i1[0], i1[1], i0[2]) - V(i0[0], i1[1], i0[2]));
    double c01 = V(i0[0], i0[1], i1[2]) + w[0] * (V(i1[0], i0[1], i1[2]) - V(i0[0], i0[1], i1[2]));
    double c11 = V(i0[0], i1[1], i1[2]) + w[0] * (V(i1[0], i1[1], i1[2]) - V(i0[0], i1[1], i1[2]));
#undef V
    double c0 = c00 + w[1] * (c10 - c00);
    double c1 = c01 + w[1] * (c11 - c01);
    return c0 + w[2] * (c1 - c0);
}

static double normalise(double v, int dtype, float lo, float hi)
{
    double s;
    if (dtype == ORC_U8) s = v / 255.0;
    else if (dtype == ORC_U16) s = v / 65535.0;
    else s = (v - (double)lo) / ((double)hi - (double)lo);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    return s;
}

typedef struct {
    const void *vol;
    int dtype, n[3];
    float vlo, vhi;
    const float *tf;
    int N;
    float dt, ref;
    int mode;
    const uint8_t *flags;
    int B, nb[3];
    const int32_t *boxes;   /* mode 2: tight box per brick, half-voxel units */
} render_ctx;

/* one pixel: writes RGBA (premultiplied) and returns the number of samples
 * composited */
static int64_t march_pixel(const render_ctx *r, const orc_camera *cam, int px, int py, double out[4])
{
    float o[3], d[3];
    ray_for_pixel(cam, px, py, o, d);
    out[0] = out[1] = out[2] = out[3] = 0.0;
    float blo[3] = {0.0f, 0.0f, 0.0f};
    float bhi[3] = {(float)r->n[0], (float)r->n[1], (float)r->n[2]};
    float tn, tx;
    if (!slab(o, d, blo, bhi, &tn, &tx)) return 0;
    float t0 = tn > 0.0f ? tn : 0.0f;
    double expo = r->ref > 0.0f ? (double)r->dt / (double)r->ref : 1.0;
    double C[3] = {0, 0, 0}, A = 0.0;
    int64_t taken = 0;
    for (int64_t k = 0;; ++k) {
        float kk = (float)k + 0.5f;
        float step = kk * r->dt;
        float t = t0 + step;
        if (!(t < tx)) break;
        float p[3];
        int inside = 1;
        for (int a = 0; a < 3; ++a) {
            float td = t * d[a];
            p[a] = o[a] + td;
            if (!(p[a] >= 0.0f && p[a] < bhi[a])) inside = 0;
        }
        if (!inside) continue;
        if (r->mode == 1 || r->mode == 2) {
            int b[3];
            for (int a = 0; a < 3; ++a) b[a] = (int)floorf(p[a]) / r->B;
            const size_t id = (size_t)b[0] + (size_t)r->nb[0] * ((size_t)b[1] + (size_t)r->nb[1] * b[2]);
            if (!r->flags[id]) continue;
            if (r->mode == 2) {
                /* only samples inside the brick's tight box (half-voxel units) */
                const int32_t *box = r->boxes + 6 * id;
                int in = 1;
                for (int a = 0; a < 3; ++a)
                    if (!(p[a] >= (float)box[a] * 0.5f && p[a] < (float)box[3 + a] * 0.5f)) in = 0;
                if (!in) continue;
            }
        }
        double s = normalise(trilinear(r->vol, r->dtype, r->n, p), r->dtype, r->vlo, r->vhi);
        double x = s * (double)(r->N - 1);
        int i0 = (int)floor(x);
        if (i0 > r->N - 2) i0 = r->N - 2;
        double f = x - (double)i0;
        double c[4];
        for (int ch = 0; ch < 4; ++ch) {
            double a0 = ch == 3 ? tf_alpha(r->tf, i0) : r->tf[4 * i0 + ch];
            double a1 = ch == 3 ? tf_alpha(r->tf, i0 + 1) : r->tf[4 * (i0 + 1) + ch];
            c[ch] = a0 + f * (a1 - a0);
        }
        double alpha = r->ref > 0.0f ? 1.0 - pow(1.0 - c[3], expo) : c[3];
        double w = (1.0 - A) * alpha;
        for (int ch = 0; ch < 3; ++ch) C[ch] += w * c[ch];
        A += w;
        ++taken;
    }
    out[0] = C[0];
    out[1] = C[1];
    out[2] = C[2];
    out[3] = A;
    return taken;
}

/* Renders either every pixel (pixels == NULL; out is [H][W][4], row 0 at the
 * top) or the listed pixels (pixels = npix (x,y) pairs; out is [npix][4]).
 * counts (optional) receives the number of composited samples per output
 * pixel.  mode 0: full march; mode 1: only samples of flagged bricks
 * (flags, B); mode 2: only samples inside the tight box of a flagged brick
 * (boxes, half-voxel units, 6 per brick). */
int orc_render(const void *vol, int dtype, int nx, int ny, int nz, float vlo, float vhi,
               const float *tf, int N, const orc_camera *cam, int W, int H, float dt, float ref,
               int mode, const uint8_t *flags, int B, const int32_t *pixels, int64_t npix,
               double *out, int64_t *counts, const int32_t *boxes)
{
    if (!vol || !tf || !cam || !out || N < 2 || W < 1 || H < 1 || !(dt > 0.0f)) return -1;
    render_ctx r = {vol, dtype, {nx, ny, nz}, vlo, vhi, tf, N, dt, ref, mode, flags, B, {0, 0, 0}, boxes};
    if (mode == 2 && !boxes) return -1;
    if (mode == 1 || mode == 2) {
        if (!flags || B < 1) return -1;
        r.nb[0] = (int)ceil_div(nx, B);
        r.nb[1] = (int)ceil_div(ny, B);
        r.nb[2] = (int)ceil_div(nz, B);
    }
    int64_t total = pixels ? npix : (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < total; ++i) {
        int px = pixels ? pixels[2 * i] : (int)(i % W);
        int py = pixels ? pixels[2 * i + 1] : (int)(i / W);
        int64_t c = march_pixel(&r, cam, px, py, out + 4 * i);
        if (counts) counts[i] = c;
    }
    return 0;
}

/* exported for the pins: the FP32 ray of one pixel, and its volume slab */
int orc_ray(const orc_camera *cam, int px, int py, float *o, float *d)
{
    ray_for_pixel(cam, px, py, o, d);
    return 0;
}

/* post-classified RGBA at one FP32 point (trilinear value, then TF lookup),
 * before opacity correction; exported for the classification pins */
int orc_sample(const void *vol, int dtype, int nx, int ny, int nz, float vlo, float vhi,
               const float *tf, int N, const float *points, int64_t npts, double *rgba)
{
    int n[3] = {nx, ny, nz};
    for (int64_t i = 0; i < npts; ++i) {
        double s = normalise(trilinear(vol, dtype, n, points + 3 * i), dtype, vlo, vhi);
        double x = s * (double)(N - 1);
        int i0 = (int)floor(x);
        if (i0 > N - 2) i0 = N - 2;
        double f = x - (double)i0;
        for (int ch = 0; ch < 4; ++ch) {
            double a0 = ch == 3 ? tf_alpha(tf, i0) : tf[4 * i0 + ch];
            double a1 = ch == 3 ? tf_alpha(tf, i0 + 1) : tf[4 * (i0 + 1) + ch];
            rgba[4 * i + ch] = a0 + f * (a1 - a0);
        }
    }
    return 0;
}

/* threads the OpenMP loops of this library use (for reporting) */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* sets the thread count of the OpenMP loops (n >= 1; for timing only) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
