// render.hip -- ray marching with empty-space skipping (Sec. 3, Sec. 4.1).
//
// Emission-absorption, post-classification (interpolate, then look up the
// TF), no gradient shading, no early ray termination.  One lane per pixel,
// one workgroup per 8x8 pixel tile; a long tile splits each ray's samples
// into two consecutive segments, one per wave, combined front to back.
//
// Every accelerator visits a subset of one global sample lattice per ray,
// t_k = t0 + (k+1/2) dt, and only ever drops samples that lie in empty
// bricks (alpha exactly 0); every mode splits a tile the same way, so every
// mode produces the same image as the full march, bit for bit:
//  - NONE: every k with t_k < t_exit whose point lies in [0,n)^3.
//  - GRID: the same loop, but a sample in an empty macrocell (= brick) jumps
//    to the last sample still inside that brick.  Sample points are
//    monotone per component in k, so if the first and the last sample of the
//    jump lie in the same brick, so do all samples between them.
//  - LBVH / KD: ordered traversal (near child first by the sign of the ray
//    direction along the node's split axis; children are separated by that
//    plane, so leaves come out in sample order).  For each leaf, a
//    conservative k range comes from an expanded slab test and each sample is
//    kept iff its point lies inside the leaf's box (half-open).  An LBVH
//    subtree whose bricks fill its box is one leaf with that box.
//  - HYBRID (Sec. 3.3): the KD traversal, but inside each leaf the samples
//    are marched with the GRID rule restricted to the leaf's box and k range,
//    so exactly the samples of non-empty bricks are composited.
//
// Geometry (ray set-up, slabs, t_k, p_k, membership) is FP32 without
// contraction: the whole file is compiled with -ffp-contract=off, and the
// value path uses explicit fmaf.
#include "esk_internal.hpp"

namespace esk {
namespace {

constexpr float kBoxEps = 1.0f / 32.0f;   // voxel-space slack of the culling tests
#ifndef ESK_MARCH_GROUP
#define ESK_MARCH_GROUP 4
#endif
constexpr int kGroup = ESK_MARCH_GROUP;   // samples gathered before compositing

struct Ray {
    float o[3], d[3];
    float inv[3];   // 1/d (0 where d == 0): conservative tests only
    float t0, tx;
    float clo, chi;   // the t range of the samples this wave marches (its segment)
    // the ray in half-voxel units (o2 = 2 o, inv2 = inv / 2): slab values
    // against half-unit box bounds equal the voxel-unit ones bit for bit
    // (scaling by 2 commutes with rounding), without converting each bound
    float o2[3], inv2[3];
};

__device__ inline void make_ray(const esk_camera &c, int px, int py, Ray &r)
{
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    float v[3];
    for (int a = 0; a < 3; ++a) {
        const float t1 = fx * c.du[a];
        const float t2 = fy * c.dv[a];
        if (c.ortho) {
            r.o[a] = (c.eye[a] + t1) + t2;
            v[a] = c.dir00[a];
        } else {
            r.o[a] = c.eye[a];
            v[a] = (c.dir00[a] + t1) + t2;
        }
    }
    const float l2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    const float len = sqrtf(l2);
    for (int a = 0; a < 3; ++a) {
        r.d[a] = v[a] / len;
        // d == 0: a huge reciprocal makes the slab unbounded when the origin
        // is inside it and empty when outside, without a branch
        r.inv[a] = r.d[a] != 0.0f ? __builtin_amdgcn_rcpf(r.d[a]) : 1.0e30f;
        r.o2[a] = r.o[a] * 2.0f;
        r.inv2[a] = r.inv[a] * 0.5f;
    }
}

// slab_fast in half-voxel units: bounds lo2/hi2 are box bounds times 2
__device__ inline void slab_half(const Ray &r, const float lo2[3], const float hi2[3], float &tn, float &tf)
{
    float t0 = -3.402823466e+38f, t1 = 3.402823466e+38f;
    for (int a = 0; a < 3; ++a) {
        const float ta = (lo2[a] - r.o2[a]) * r.inv2[a];
        const float tb = (hi2[a] - r.o2[a]) * r.inv2[a];
        t0 = fmaxf(t0, fminf(ta, tb));
        t1 = fminf(t1, fmaxf(ta, tb));
    }
    tn = t0;
    tf = t1;
}

__device__ inline bool slab(const Ray &r, const float lo[3], const float hi[3], float &tn, float &tf)
{
    float t0 = -3.402823466e+38f, t1 = 3.402823466e+38f;
    for (int a = 0; a < 3; ++a) {
        if (r.d[a] != 0.0f) {
            const float ta = (lo[a] - r.o[a]) / r.d[a];
            const float tb = (hi[a] - r.o[a]) / r.d[a];
            const float mn = ta < tb ? ta : tb;
            const float mx = ta < tb ? tb : ta;
            if (mn > t0) t0 = mn;
            if (mx < t1) t1 = mx;
        } else if (r.o[a] < lo[a] || r.o[a] >= hi[a]) {
            return false;
        }
    }
    tn = t0;
    tf = t1;
    return true;
}

// the slab test with reciprocal multiplies and no branches: only used where
// the result is widened by a margin and every sample is then checked exactly
__device__ inline void slab_fast(const Ray &r, const float lo[3], const float hi[3], float &tn, float &tf)
{
    float t0 = -3.402823466e+38f, t1 = 3.402823466e+38f;
    for (int a = 0; a < 3; ++a) {
        const float ta = (lo[a] - r.o[a]) * r.inv[a];
        const float tb = (hi[a] - r.o[a]) * r.inv[a];
        t0 = fmaxf(t0, fminf(ta, tb));
        t1 = fminf(t1, fmaxf(ta, tb));
    }
    tn = t0;
    tf = t1;
}

__device__ inline float lattice_t(const Ray &r, float dt, int k)
{
    const float kk = (float)k + 0.5f;
    const float step = kk * dt;
    return r.t0 + step;
}

__device__ inline void point_at(const Ray &r, float t, float p[3])
{
    for (int a = 0; a < 3; ++a) {
        const float td = t * r.d[a];
        p[a] = r.o[a] + td;
    }
}

struct Accum {
    float c[3], a;
    int n;
};

struct Vol {
    int n[3];
    float fn[3];
    float fm[3];       // n - 1: the largest continuous voxel index
    uint32_t nq0, nq1; // blocks along x and y
};

// cell-centred trilinear interpolation (clamp to edge) from the blocked copy:
// voxel (x, y, z) of stored block ((z>>3)*nq1 + (y>>3))*nq0 + (x>>3) sits at
// ((z&7)*9 + (y&7))*9 + (x&7), and its +1 neighbours at +1, +9, +81.  The
// continuous index u = p - 1/2 is clamped to [0, n-1] per axis: there the
// weight of the far neighbour is 0, so the result equals clamping both
// neighbour indices to the volume, and any point gives valid addresses.
// Split in two so a group of samples can issue all its gathers before the
// first interpolation: gather() loads the 8 corners and the weights, lerp3()
// combines them.
struct Corners {
    float c[8];
    float w[3];
};

template <typename T, typename IDX>
__device__ inline void gather(const T *__restrict__ vol, const Vol &v, const float p[3], Corners &g)
{
    const float ux = fminf(fmaxf(p[0] - 0.5f, 0.0f), v.fm[0]);
    const float uy = fminf(fmaxf(p[1] - 0.5f, 0.0f), v.fm[1]);
    const float uz = fminf(fmaxf(p[2] - 0.5f, 0.0f), v.fm[2]);
    const float fx = floorf(ux), fy = floorf(uy), fz = floorf(uz);
    g.w[0] = ux - fx;
    g.w[1] = uy - fy;
    g.w[2] = uz - fz;
    const uint32_t ix = (uint32_t)(int)fx, iy = (uint32_t)(int)fy, iz = (uint32_t)(int)fz;
    // indices are below 32768, block counts below 4096 (the masks state it),
    // so the 24-bit multiplies are exact; IDX = uint32_t: the copy is
    // < 4 GiB, so byte offsets are 32-bit and every load is a scalar base
    // plus one 32-bit vector offset
    constexpr uint32_t E = (uint32_t)sizeof(T);
    const uint32_t row = __umul24((iz >> 3) & 0xfffu, v.nq1 & 0xfffu) + ((iy >> 3) & 0xfffu);
    const uint32_t local = __umul24(__umul24(iz & 7u, 9u) + (iy & 7u), 9u) + (ix & 7u);
    IDX off;
    if constexpr (sizeof(IDX) == 4)
        off = __umul24(__umul24(row, v.nq0 & 0xfffu) + ((ix >> 3) & 0xfffu), (uint32_t)kSwzBlock * E) + local * E;
    else
        off = ((IDX)row * v.nq0 + ((ix >> 3) & 0xfffu)) * ((IDX)kSwzBlock * E) + (IDX)(local * E);
    const char *__restrict__ base = reinterpret_cast<const char *>(vol) + off;
    if constexpr (sizeof(T) == 4) {
        // x and x + 1 are adjacent: one 8-byte (dword-aligned) load per row
        auto ld2 = [&](uint32_t o, float &a, float &b) {
            float q[2];
            __builtin_memcpy(q, base + o, 8);
            a = q[0];
            b = q[1];
        };
        ld2(0, g.c[0], g.c[1]);
        ld2(9 * E, g.c[2], g.c[3]);
        ld2(81 * E, g.c[4], g.c[5]);
        ld2(90 * E, g.c[6], g.c[7]);
    } else {
        auto ld = [&](uint32_t o) { return (float)*reinterpret_cast<const T *>(base + o); };
        g.c[0] = ld(0);
        g.c[1] = ld(E);
        g.c[2] = ld(9 * E);
        g.c[3] = ld(10 * E);
        g.c[4] = ld(81 * E);
        g.c[5] = ld(82 * E);
        g.c[6] = ld(90 * E);
        g.c[7] = ld(91 * E);
    }
}

__device__ inline float lerp3(const Corners &g)
{
    const float wx = g.w[0], wy = g.w[1], wz = g.w[2];
    const float c00 = fmaf(wx, g.c[1] - g.c[0], g.c[0]), c10 = fmaf(wx, g.c[3] - g.c[2], g.c[2]);
    const float c01 = fmaf(wx, g.c[5] - g.c[4], g.c[4]), c11 = fmaf(wx, g.c[7] - g.c[6], g.c[6]);
    const float c0 = fmaf(wy, c10 - c00, c00), c1 = fmaf(wy, c11 - c01, c01);
    return fmaf(wz, c1 - c0, c0);
}

template <typename T, typename IDX>
__device__ inline float trilinear(const T *__restrict__ vol, const Vol &v, const float p[3])
{
    Corners g;
    gather<T, IDX>(vol, v, p, g);
    return lerp3(g);
}

// keeps the scheduler from interleaving a group's gathers with its arithmetic
__device__ inline void group_fence() { __builtin_amdgcn_sched_barrier(0); }

struct Shade {
    const float4 *tf;
    int N;
    float vlo, vscale, expo;
    int correct;
};

// post-classification + opacity correction + front-to-back "over".  With
// ok == false the sample contributes nothing (opacity 0: colour and alpha
// stay bit-identical) and is not counted, so callers can run a fixed group
// of samples without branching per sample.
__device__ inline void composite(const Shade &s, float v, bool ok, Accum &acc)
{
    float x = (v - s.vlo) * s.vscale;
    x = fminf(fmaxf(x, 0.0f), 1.0f) * (float)(s.N - 1);
    const int i0 = min((int)x, s.N - 2);
    const float f = x - (float)i0;
    const float4 a = s.tf[i0], b = s.tf[i0 + 1];
    const float r = fmaf(f, b.x - a.x, a.x);
    const float g = fmaf(f, b.y - a.y, a.y);
    const float bl = fmaf(f, b.z - a.z, a.z);
    float al = fmaf(f, b.w - a.w, a.w);
    if (s.correct) {
        // 1 - (1-a)^(dt/ref); exactly 0 for a == 0
        const float l = __builtin_amdgcn_logf(1.0f - al);
        const float e = __builtin_amdgcn_exp2f(s.expo * l);
        al = al > 0.0f ? 1.0f - e : 0.0f;
    }
    al = ok ? al : 0.0f;
    const float w = (1.0f - acc.a) * al;
    acc.c[0] = fmaf(w, r, acc.c[0]);
    acc.c[1] = fmaf(w, g, acc.c[1]);
    acc.c[2] = fmaf(w, bl, acc.c[2]);
    acc.a = acc.a + w;
    acc.n += ok ? 1 : 0;
}

__device__ inline bool inside(const Vol &v, const float p[3])
{
    // non-short-circuit: one mask, no branch per axis
    return (p[0] >= 0.0f) & (p[0] < v.fn[0]) & (p[1] >= 0.0f) & (p[1] < v.fn[1]) & (p[2] >= 0.0f) &
           (p[2] < v.fn[2]);
}

// conservative hit of a box [lo/2, hi/2) (bounds in half-voxel units) by the ray segment
__device__ inline bool hit_box(const Ray &r, float dt, const int lo[3], const int hi[3])
{
    float l[3], h[3];
    for (int a = 0; a < 3; ++a) {
        l[a] = (float)lo[a] - 2.0f * kBoxEps;
        h[a] = (float)hi[a] + 2.0f * kBoxEps;
    }
    float tn, tf;
    slab_half(r, l, h, tn, tf);
    return tn <= tf + dt && tf >= r.clo - dt && tn <= r.chi + dt;
}

struct GridRef {
    const uint32_t *bits;   // one bit per brick, linear brick id
    int sh, B;              // log2 of the brick edge, brick edge
    uint32_t nbx, nby;      // bricks along x and y
    int n[3];
};

__device__ inline GridRef grid_ref(const RenderArgs &ra)
{
    GridRef g;
    g.bits = ra.grid;
    g.sh = ra.vol.log2B;
    g.B = ra.vol.B;
    // < 2^28 bricks, at most 1024 per axis: 32-bit ids, 24-bit multiplies
    g.nbx = (uint32_t)ra.vol.nb[0] & 0x7ffu;
    g.nby = (uint32_t)ra.vol.nb[1] & 0x7ffu;
    g.n[0] = ra.vol.nx;
    g.n[1] = ra.vol.ny;
    g.n[2] = ra.vol.nz;
    return g;
}

// Macrocell-grid march (macrocell = brick) over the samples k in [k, k_end)
// whose points lie in the box [lo, hi) of the volume: a sample in an empty
// brick jumps to the last sample inside that brick (sample points are
// monotone per component, so every sample between lies in the brick too);
// in a non-empty brick a group of samples from k is composited, and those
// in the brick (and the box) are consecutive and start with k, so k
// advances by their count.  The whole ray with the volume as the box is the
// grid accelerator; a k-d leaf's sample range and box is the hybrid grid.
template <typename T, typename IDX>
__device__ inline void march_grid(const Ray &r, float dt, int k, int k_end, const float lo[3], const float hi[3],
                                  const GridRef &gr, const T *__restrict__ vol, const Vol &v, const Shade &s,
                                  Accum &acc)
{
    const int sh = gr.sh, B = gr.B;
    while (k < k_end) {
        const float t = lattice_t(r, dt, k);
        if (!(t < r.tx)) break;
        float p[3];
        point_at(r, t, p);
        if (!((p[0] >= lo[0]) & (p[0] < hi[0]) & (p[1] >= lo[1]) & (p[1] < hi[1]) & (p[2] >= lo[2]) &
              (p[2] < hi[2]))) {
            ++k;
            continue;
        }
        const int bx = (int)p[0] >> sh, by = (int)p[1] >> sh, bz = (int)p[2] >> sh;
        const uint32_t b = (uint32_t)bx + __umul24(gr.nbx, (uint32_t)by + __umul24(gr.nby, (uint32_t)bz));
        const float blo[3] = {(float)(bx << sh), (float)(by << sh), (float)(bz << sh)};
        const float bhi[3] = {(float)min((bx << sh) + B, gr.n[0]), (float)min((by << sh) + B, gr.n[1]),
                              (float)min((bz << sh) + B, gr.n[2])};
        if ((gr.bits[b >> 5] >> (b & 31)) & 1u) {
            const float ml[3] = {fmaxf(blo[0], lo[0]), fmaxf(blo[1], lo[1]), fmaxf(blo[2], lo[2])};
            const float mh[3] = {fminf(bhi[0], hi[0]), fminf(bhi[1], hi[1]), fminf(bhi[2], hi[2])};
            Corners g[kGroup];
            bool ok[kGroup];
            int taken = 0;
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                const float tj = lattice_t(r, dt, k + j);
                float q[3];
                point_at(r, tj, q);
                ok[j] = (k + j < k_end) & (tj < r.tx) & (q[0] >= ml[0]) & (q[0] < mh[0]) & (q[1] >= ml[1]) &
                        (q[1] < mh[1]) & (q[2] >= ml[2]) & (q[2] < mh[2]);
                gather<T, IDX>(vol, v, q, g[j]);
                taken += ok[j] ? 1 : 0;
            }
            group_fence();
#pragma unroll
            for (int j = 0; j < kGroup; ++j) composite(s, lerp3(g[j]), ok[j], acc);
            k += taken;
            continue;
        }
        // empty macrocell: jump to the last sample inside it
        float cn, cx;
        int next = k + 1;
        slab_fast(r, blo, bhi, cn, cx);
        float fj = (cx - r.t0) * __builtin_amdgcn_rcpf(dt) - 0.5f;
        fj = fminf(fmaxf(fj, -4.0f), 1.0e9f);
        const int kj = (int)floorf(fj);
        for (int c = kj; c >= kj - 1; --c) {
            if (c <= k) break;
            float q[3];
            point_at(r, lattice_t(r, dt, c), q);
            if (inside(v, q) && ((int)q[0] >> sh) == bx && ((int)q[1] >> sh) == by && ((int)q[2] >> sh) == bz) {
                next = c + 1;
                break;
            }
        }
        k = next;
    }
}

// The sample range [ka, kb) that may fall in the leaf box [lo/2, hi/2)
// (conservative: membership is decided per sample against bl/bh, the box in
// voxels); an empty range where the ray misses the box.
__device__ inline void leaf_range(const Ray &r, float dt, const int lo[3], const int hi[3], int &ka, int &kb,
                                  float bl[3], float bh[3])
{
    float l[3], h[3];
    for (int a = 0; a < 3; ++a) {
        bl[a] = (float)lo[a] * 0.5f;   // half-voxel units: exact
        bh[a] = (float)hi[a] * 0.5f;
        l[a] = (float)lo[a] - 2.0f * kBoxEps;
        h[a] = (float)hi[a] + 2.0f * kBoxEps;
    }
    float tn, tf;
    slab_half(r, l, h, tn, tf);
    ka = kb = 0;
    if (tn > tf + dt) return;
    const float idt = __builtin_amdgcn_rcpf(dt);
    float fa = (tn - r.t0) * idt - 0.5f;
    float fb = (tf - r.t0) * idt - 0.5f;
    fa = fminf(fmaxf(fa, -4.0f), 1.0e9f);
    fb = fminf(fmaxf(fb, -4.0f), 1.0e9f);
    // Along the ray the box slack kBoxEps is at least 1/32 voxel, and the
    // FP32 error of tn, tf (and of fa, fb, in voxels) stays below t * 2^-21:
    // under 1/32 voxel while t < 65536, for any dt.  Rays that end before
    // t = 16384 therefore take [floor(fa), floor(fb) + 1) as is; farther
    // ones widen it by a sample on each side.
    const int m = r.tx < 16384.0f ? 0 : 1;
    ka = max(0, (int)floorf(fa) - m);
    kb = (int)floorf(fb) + 1 + m;
}

// samples of the lattice that fall in the leaf box [lo/2, hi/2), found with
// the macrocell grid (hybrid grid): only those in non-empty bricks
template <typename T, typename IDX>
__device__ inline void march_leaf_grid(const Ray &r, float dt, int ks, int ke, const int lo[3], const int hi[3],
                                       const GridRef &gr, const T *__restrict__ vol, const Vol &v, const Shade &s,
                                       Accum &acc)
{
    int ka, kb;
    float bl[3], bh[3];
    leaf_range(r, dt, lo, hi, ka, kb, bl, bh);
    ka = max(ka, ks);
    kb = min(kb, ke);
    if (ka < kb) march_grid<T, IDX>(r, dt, ka, kb, bl, bh, gr, vol, v, s, acc);
}

__device__ inline void unpack_box(uint32_t w0, uint32_t w1, uint32_t w2, int lo[3], int hi[3])
{
    lo[0] = (int)(w0 & 0xffffu);
    lo[1] = (int)(w0 >> 16);
    lo[2] = (int)(w1 & 0xffffu);
    hi[0] = (int)(w1 >> 16);
    hi[1] = (int)(w2 & 0xffffu);
    hi[2] = (int)(w2 >> 16);
}

// Where a lane stands in its ordered traversal: cur is still to be visited
// while `have` holds; sp entries wait on the lane's LDS stack.
struct Trav {
    uint32_t cur;
    bool have;
    int sp;
};

// Ordered traversal of a binary hierarchy stored as RNode records (LBVH or
// k-d): near child first by the sign of the direction along the node's
// split axis, far child on the wave's LDS stack (lane-interleaved).  Descends to the
// lane's next leaf (lo/hi: its box; popped leaves fetch their packed box);
// false once the hierarchy is exhausted.
__device__ inline bool next_leaf(const Ray &r, float dt, const RNode *__restrict__ nodes,
                                 const uint4 *__restrict__ leafbox, int *stk, int cap, Trav &tr, int lo[3],
                                 int hi[3])
{
    while (true) {
        if (!tr.have) {
            if (tr.sp == 0) return false;
            --tr.sp;
            tr.cur = (uint32_t)stk[tr.sp * 64 + (threadIdx.x & 63)];
            if (tr.cur & kLeaf) {
                const uint4 b = leafbox[tr.cur & kIndexMask];
                unpack_box(b.x, b.y, b.z, lo, hi);
            }
            tr.have = true;
        }
        if (tr.cur & kLeaf) {
            tr.have = false;
            return true;
        }
        const uint4 *q = reinterpret_cast<const uint4 *>(&nodes[tr.cur & kIndexMask]);
        const uint4 A = q[0], Q = q[1];
        int l0[3], h0[3], l1[3], h1[3];
        unpack_box(A.x, A.y, A.z, l0, h0);
        unpack_box(A.w, Q.x, Q.y, l1, h1);
        const uint32_t c0 = Q.z & (kLeaf | kIndexMask), c1 = Q.w;
        const int axis = (int)((Q.z >> 29) & 3u);
        const bool hit0 = hit_box(r, dt, l0, h0), hit1 = hit_box(r, dt, l1, h1);
        // select, not index: a dynamic index would move the ray to scratch
        const float da = axis == 0 ? r.d[0] : (axis == 1 ? r.d[1] : r.d[2]);
        const bool flip = da < 0.0f;
        const bool hn = flip ? hit1 : hit0, hf = flip ? hit0 : hit1;
        const uint32_t nr = flip ? c1 : c0, fr = flip ? c0 : c1;
        if (hn || hf) {
            if (hn && hf && tr.sp < cap) {
                stk[tr.sp * 64 + (threadIdx.x & 63)] = (int)fr;
                ++tr.sp;
            }
            tr.cur = hn ? nr : fr;
            const bool one = hn == flip;   // child 1 taken
            for (int a = 0; a < 3; ++a) {
                lo[a] = one ? l1[a] : l0[a];
                hi[a] = one ? h1[a] : h0[a];
            }
        } else {
            tr.have = false;
        }
    }
}

// The tree renders: each round every lane descends to its next two leaves
// (lanes that hold them wait, so the wave's descents run together), then
// marches their samples as one sequence in groups -- leaf one's range, then
// leaf two's, in ray order -- so a round costs the wave its longest pair of
// leaves rather than its longest leaf twice (measured: three or four leaves
// per round gain nothing more).  HYB: each leaf is marched with the
// macrocell grid inside it (hybrid grid).
template <typename T, typename IDX, bool HYB>
__device__ inline void traverse(const Ray &r, float dt, int ks, int ke, const RNode *__restrict__ nodes,
                                const uint4 *__restrict__ leafbox, const GridRef &gr, uint32_t root, int lo[3], int hi[3],
                                int *stk, int cap, const T *__restrict__ vol, const Vol &v, const Shade &s,
                                Accum &acc)
{
    if (!hit_box(r, dt, lo, hi)) return;
    Trav tr{root, true, 0};
    while (true) {
        if (!next_leaf(r, dt, nodes, leafbox, stk, cap, tr, lo, hi)) return;
        int lo2[3], hi2[3];
        const bool two = next_leaf(r, dt, nodes, leafbox, stk, cap, tr, lo2, hi2);
        if constexpr (HYB) {
            march_leaf_grid<T, IDX>(r, dt, ks, ke, lo, hi, gr, vol, v, s, acc);
            if (two) march_leaf_grid<T, IDX>(r, dt, ks, ke, lo2, hi2, gr, vol, v, s, acc);
        } else {
            int ka1, kb1, ka2 = 0, kb2 = 0;
            float bl1[3], bh1[3], bl2[3] = {0.0f, 0.0f, 0.0f}, bh2[3] = {0.0f, 0.0f, 0.0f};
            leaf_range(r, dt, lo, hi, ka1, kb1, bl1, bh1);
            if (two) leaf_range(r, dt, lo2, hi2, ka2, kb2, bl2, bh2);
            // the wave's segment of the sample sequence
            ka1 = max(ka1, ks);
            kb1 = min(kb1, ke);
            ka2 = max(ka2, ks);
            kb2 = min(kb2, ke);
            const int n1 = max(0, kb1 - ka1), n = n1 + max(0, kb2 - ka2);
            for (int i = 0; i < n; i += kGroup) {
                // a group of the sequence: the points first, then every
                // gather (the clamped addresses are valid for any point),
                // then the group is composited in order
                Corners g[kGroup];
                bool ok[kGroup];
                float p[kGroup][3];
#pragma unroll
                for (int j = 0; j < kGroup; ++j) {
                    const int idx = i + j;
                    const bool first = idx < n1;
                    const int k = first ? ka1 + idx : ka2 + (idx - n1);
                    const float t = lattice_t(r, dt, k);
                    point_at(r, t, p[j]);
                    bool in = (idx < n) & (t < r.tx);
                    for (int a = 0; a < 3; ++a)
                        in = in & (p[j][a] >= (first ? bl1[a] : bl2[a])) & (p[j][a] < (first ? bh1[a] : bh2[a]));
                    ok[j] = in;
                }
                group_fence();
#pragma unroll
                for (int j = 0; j < kGroup; ++j) gather<T, IDX>(vol, v, p[j], g[j]);
                group_fence();
#pragma unroll
                for (int j = 0; j < kGroup; ++j) composite(s, lerp3(g[j]), ok[j], acc);
            }
        }
        if (!two) return;
    }
}

// Waves per SIMD the render kernels are compiled for.  The scheduler
// otherwise trades latency hiding for occupancy: aiming at 5-8 waves it
// waits on each sample's gathers in turn instead of issuing a whole group
// before the first wait (measured 20-40 % slower marches).  2 for the full
// march, 4 for the others (with two-wave tiles: measured best of 2..6; 3
// and 4 for the full march measured the same or slower).
constexpr int render_waves_for(int accel) { return accel == ESK_ACCEL_NONE ? 2 : 4; }

// One 8x8-pixel tile (tbx, tby) of one request.  TFL: the TF (N <= 1024
// entries) is staged in LDS; otherwise read from global memory.
//
// Every wave computes the tile's rays and K, the lattice samples before the
// exit of its longest ray; the tile takes S = clamp(K / seg_len, 1, max)
// waves and the others end at once.  Wave j marches the samples
// [K_r j / S, K_r (j + 1) / S) of each ray r (the last wave to the ray's
// end) in any mode, from zero colour and opacity; wave 0 then combines the
// partial results front to back.  K depends on the camera and the volume
// only, so every mode splits a tile the same way and every skipping mode
// still reproduces the full march bit for bit.
template <int ACCEL, typename T, typename IDX, bool TFL>
__device__ inline void render_tile(const RenderArgs &ra, int tbx, int tby)
{
    extern __shared__ float4 lds[];
    constexpr int kSegMax = kRaySegments;
    __shared__ float4 part_c[kSegMax > 1 ? kSegMax - 1 : 1][64];
    __shared__ int part_n[kSegMax > 1 ? kSegMax - 1 : 1][64];
    constexpr bool tf_lds = TFL;

    const int lane = threadIdx.x & 63;
    // wave-uniform (scalar) values: whole waves leave or branch together
    const int seg = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int px = tbx * 8 + (lane & 7);
    const int py = tby * 8 + (lane >> 3);
    const bool live = px < ra.W && py < ra.H;

    Vol v;
    v.n[0] = ra.vol.nx; v.n[1] = ra.vol.ny; v.n[2] = ra.vol.nz;
    for (int a = 0; a < 3; ++a) {
        v.fn[a] = (float)v.n[a];
        v.fm[a] = (float)(v.n[a] - 1);
    }
    v.nq0 = (uint32_t)ra.vol.nq[0];
    v.nq1 = (uint32_t)ra.vol.nq[1];
    const float dt = ra.dt;

    Ray r;
    make_ray(ra.cam, px, py, r);
    const float zero[3] = {0.0f, 0.0f, 0.0f};
    float tn = 0.0f, tx = 0.0f;
    const bool hit = live && slab(r, zero, v.fn, tn, tx);
    r.t0 = hit ? (tn > 0.0f ? tn : 0.0f) : 0.0f;
    r.tx = hit ? tx : 0.0f;
    int K = 0;
    if (hit) K = (int)fminf(fmaxf((r.tx - r.t0) * __builtin_amdgcn_rcpf(dt), 0.0f), 1.0e9f);
    int kmax = K;
    for (int o = 32; o >= 1; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const int S = __builtin_amdgcn_readfirstlane(min(kSegMax, max(1, kmax / ra.seg_len)));
    if (seg >= S) return;

    if (tf_lds) {
        const float4 *src = reinterpret_cast<const float4 *>(ra.tf);
        for (int i = threadIdx.x; i < ra.N; i += 64 * S) lds[i] = src[i];
        __syncthreads();
    }
    int *stk = reinterpret_cast<int *>(lds + (tf_lds ? ra.N : 0)) + seg * ra.stack_cap * 64;

    const T *__restrict__ vol = static_cast<const T *>(ra.vol.swz);
    Shade s;
    s.tf = tf_lds ? lds : reinterpret_cast<const float4 *>(ra.tf);
    s.N = ra.N;
    s.vlo = ra.vlo;
    s.vscale = ra.vscale;
    s.expo = ra.expo;
    s.correct = ra.correct;

    // this wave's samples [ks, ke) and their t range (culling slack covers rounding)
    const int ks = (int)(((int64_t)K * seg) / S);
    const int ke = seg == S - 1 ? (1 << 30) : (int)(((int64_t)K * (seg + 1)) / S);
    r.clo = fmaf((float)ks, dt, r.t0);
    r.chi = seg == S - 1 ? r.tx : fmaf((float)ke, dt, r.t0);

    Accum acc = {{0.0f, 0.0f, 0.0f}, 0.0f, 0};
    if (hit) {
        if (ACCEL == ESK_ACCEL_NONE) {
            for (int k = ks;; k += kGroup) {
                Corners g[kGroup];
                bool ok[kGroup];
                bool more = true;
#pragma unroll
                for (int j = 0; j < kGroup; ++j) {
                    const float t = lattice_t(r, dt, k + j);
                    float p[3];
                    point_at(r, t, p);
                    const bool in_seg = (t < r.tx) & (k + j < ke);
                    ok[j] = in_seg & inside(v, p);
                    gather<T, IDX>(vol, v, p, g[j]);
                    more = in_seg;
                }
                group_fence();
#pragma unroll
                for (int j = 0; j < kGroup; ++j) composite(s, lerp3(g[j]), ok[j], acc);
                if (!more) break;
            }
        } else if (ACCEL == ESK_ACCEL_GRID) {
            const float zero3[3] = {0.0f, 0.0f, 0.0f};
            march_grid<T, IDX>(r, dt, ks, ke, zero3, v.fn, grid_ref(ra), vol, v, s, acc);
        } else if (ACCEL == ESK_ACCEL_LBVH) {
            const int N = (int)ra.hdr->n;
            if (N > 0) {
                int lo[3], hi[3];
                const uint4 b = ra.lb_root[0];
                unpack_box(b.x, b.y, b.z, lo, hi);
                traverse<T, IDX, false>(r, dt, ks, ke, ra.lb_rnode, ra.lb_leafbox, grid_ref(ra), N == 1 ? kLeaf : 0u,
                                        lo, hi, stk, ra.stack_cap, vol, v, s, acc);
            }
        } else if (ACCEL == ESK_ACCEL_KD || ACCEL == ESK_ACCEL_HYBRID) {
            const int M = (int)ra.hdr->kd_count;
            if (M > 0) {
                int lo[3], hi[3];
                const uint4 b = ra.kd_box[0];
                unpack_box(b.x, b.y, b.z, lo, hi);
                traverse<T, IDX, ACCEL == ESK_ACCEL_HYBRID>(r, dt, ks, ke, ra.kd_rnode, ra.kd_box, grid_ref(ra),
                                                            M == 1 ? kLeaf : 0u, lo, hi, stk, ra.stack_cap, vol, v,
                                                            s, acc);
            }
        }
    }
    if (kSegMax > 1 && S > 1) {
        if (seg > 0) {
            part_c[seg - 1][lane] = make_float4(acc.c[0], acc.c[1], acc.c[2], acc.a);
            part_n[seg - 1][lane] = acc.n;
        }
        __syncthreads();
        if (seg > 0) return;
        for (int j = 1; j < S; ++j) {
            const float4 q = part_c[j - 1][lane];
            const float t = 1.0f - acc.a;
            acc.c[0] = fmaf(t, q.x, acc.c[0]);
            acc.c[1] = fmaf(t, q.y, acc.c[1]);
            acc.c[2] = fmaf(t, q.z, acc.c[2]);
            acc.a = fmaf(t, q.w, acc.a);
            acc.n += part_n[j - 1][lane];
        }
    }
    if (!live) return;
    const int64_t pix = (int64_t)py * ra.W + px;
    reinterpret_cast<float4 *>(ra.out)[pix] = make_float4(acc.c[0], acc.c[1], acc.c[2], acc.a);
    if (ra.count) ra.count[pix] = acc.n;
}

// The i-th of the n indices [0, n) in the order c, c + 1, c - 1, c + 2,
// c - 2, ..., then the rest of the longer side: workgroups are dispatched in
// block order, so tiles start from the centre tile outwards (rows, and
// within a row columns).
__device__ inline int centre_out(int i, int c, int n)
{
    const int m = min(c, n - 1 - c);
    if (i <= 2 * m) {
        const int h = (i + 1) >> 1;
        return (i & 1) ? c + h : c - h;
    }
    const int rest = i - 2 * m;
    return c - m == 0 ? c + m + rest : c - m - rest;
}

template <int ACCEL, typename T, typename IDX, bool TFL>
__global__ __launch_bounds__(render_threads_for(ACCEL)) __attribute__((amdgpu_waves_per_eu(1, render_waves_for(ACCEL)))) void
k_render(RenderArgs ra)
{
    // block order spreads consecutive tiles round-robin over the XCDs, which
    // balances the very uneven per-tile work (giving each XCD a band of
    // tiles was measured 1.5-2x slower)
    render_tile<ACCEL, T, IDX, TFL>(ra, centre_out((int)blockIdx.x, ra.ctx, (int)gridDim.x),
                                    centre_out((int)blockIdx.y, ra.cty, (int)gridDim.y));
}

// Many requests in one launch: blockIdx.z picks the request, whose tiles
// cover the front of the (max-sized) grid; the rest of its blocks exit.
template <int ACCEL, typename T, typename IDX, bool TFL>
__global__ __launch_bounds__(render_threads_for(ACCEL)) __attribute__((amdgpu_waves_per_eu(1, render_waves_for(ACCEL)))) void
k_render_batch(const RenderArgs *__restrict__ args)
{
    const RenderArgs ra = args[blockIdx.z];
    const int ntx = (ra.W + 7) / 8, nty = (ra.H + 7) / 8;
    if ((int)blockIdx.x >= ntx || (int)blockIdx.y >= nty) return;  // uniform per block
    render_tile<ACCEL, T, IDX, TFL>(ra, centre_out((int)blockIdx.x, ra.ctx, ntx), centre_out((int)blockIdx.y, ra.cty, nty));
}

template <int ACCEL, typename T, typename IDX, bool TFL>
hipError_t launch_batch_inst(const RenderArgs *d_args, const dim3 &grid, size_t lds, hipStream_t s)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_render_batch<ACCEL, T, IDX, TFL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_render_batch<ACCEL, T, IDX, TFL>), grid, dim3(render_threads_for(ACCEL)), lds, s, d_args);
    return hipGetLastError();
}

template <int ACCEL, typename T>
hipError_t launch_batch_accel(const RenderArgs *d_args, const dim3 &grid, size_t lds, bool narrow, bool tfl,
                              hipStream_t s)
{
    if (narrow)
        return tfl ? launch_batch_inst<ACCEL, T, uint32_t, true>(d_args, grid, lds, s)
                   : launch_batch_inst<ACCEL, T, uint32_t, false>(d_args, grid, lds, s);
    return tfl ? launch_batch_inst<ACCEL, T, uint64_t, true>(d_args, grid, lds, s)
               : launch_batch_inst<ACCEL, T, uint64_t, false>(d_args, grid, lds, s);
}

template <typename T>
hipError_t launch_batch_typed(int accel, const RenderArgs *d_args, const dim3 &grid, size_t lds, bool narrow,
                              bool tfl, hipStream_t s)
{
    switch (accel) {
    case ESK_ACCEL_NONE: return launch_batch_accel<ESK_ACCEL_NONE, T>(d_args, grid, lds, narrow, tfl, s);
    case ESK_ACCEL_GRID: return launch_batch_accel<ESK_ACCEL_GRID, T>(d_args, grid, lds, narrow, tfl, s);
    case ESK_ACCEL_LBVH: return launch_batch_accel<ESK_ACCEL_LBVH, T>(d_args, grid, lds, narrow, tfl, s);
    case ESK_ACCEL_KD: return launch_batch_accel<ESK_ACCEL_KD, T>(d_args, grid, lds, narrow, tfl, s);
    case ESK_ACCEL_HYBRID: return launch_batch_accel<ESK_ACCEL_HYBRID, T>(d_args, grid, lds, narrow, tfl, s);
    }
    return hipErrorInvalidValue;
}

template <int ACCEL, typename T>
hipError_t launch_accel(const RenderArgs &r, hipStream_t s)
{
    constexpr int tile = render_tile_for(ACCEL);
    const dim3 grid((r.W + tile - 1) / tile, (r.H + tile - 1) / tile);
    const size_t lds = render_lds_bytes(ACCEL, r.N, r.N <= 1024, r.stack_cap);
    const int64_t nbytes = swz_bytes(r.vol.nq, (int)sizeof(T));
    const bool narrow = nbytes < (int64_t)0xffffffffLL;
    const bool tfl = r.N <= 1024;
    const void *fn;
    if (narrow)
        fn = tfl ? reinterpret_cast<const void *>(&k_render<ACCEL, T, uint32_t, true>)
                 : reinterpret_cast<const void *>(&k_render<ACCEL, T, uint32_t, false>);
    else
        fn = tfl ? reinterpret_cast<const void *>(&k_render<ACCEL, T, uint64_t, true>)
                 : reinterpret_cast<const void *>(&k_render<ACCEL, T, uint64_t, false>);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (narrow) {
        if (tfl) hipLaunchKernelGGL((k_render<ACCEL, T, uint32_t, true>), grid, dim3(render_threads_for(ACCEL)), lds, s, r);
        else hipLaunchKernelGGL((k_render<ACCEL, T, uint32_t, false>), grid, dim3(render_threads_for(ACCEL)), lds, s, r);
    } else {
        if (tfl) hipLaunchKernelGGL((k_render<ACCEL, T, uint64_t, true>), grid, dim3(render_threads_for(ACCEL)), lds, s, r);
        else hipLaunchKernelGGL((k_render<ACCEL, T, uint64_t, false>), grid, dim3(render_threads_for(ACCEL)), lds, s, r);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(int accel, const RenderArgs &r, hipStream_t s)
{
    switch (accel) {
    case ESK_ACCEL_NONE: return launch_accel<ESK_ACCEL_NONE, T>(r, s);
    case ESK_ACCEL_GRID: return launch_accel<ESK_ACCEL_GRID, T>(r, s);
    case ESK_ACCEL_LBVH: return launch_accel<ESK_ACCEL_LBVH, T>(r, s);
    case ESK_ACCEL_KD: return launch_accel<ESK_ACCEL_KD, T>(r, s);
    case ESK_ACCEL_HYBRID: return launch_accel<ESK_ACCEL_HYBRID, T>(r, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_render_batch(int accel, int dtype, const RenderArgs *d_args, int n, int tiles_x, int tiles_y,
                               size_t lds, bool narrow, bool tfl, hipStream_t s)
{
    const dim3 grid((unsigned)tiles_x, (unsigned)tiles_y, (unsigned)n);
    switch (dtype) {
    case ESK_U8: return launch_batch_typed<uint8_t>(accel, d_args, grid, lds, narrow, tfl, s);
    case ESK_U16: return launch_batch_typed<uint16_t>(accel, d_args, grid, lds, narrow, tfl, s);
    case ESK_F16: return launch_batch_typed<_Float16>(accel, d_args, grid, lds, narrow, tfl, s);
    case ESK_F32: return launch_batch_typed<float>(accel, d_args, grid, lds, narrow, tfl, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_render(int accel, const RenderArgs &r, hipStream_t s)
{
    switch (r.vol.dtype) {
    case ESK_U8: return launch_typed<uint8_t>(accel, r, s);
    case ESK_U16: return launch_typed<uint16_t>(accel, r, s);
    case ESK_F16: return launch_typed<_Float16>(accel, r, s);
    case ESK_F32: return launch_typed<float>(accel, r, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace esk
