// kdtree.hip -- binned k-d tree over brick occupancy (Sec. 3.2, 3.2.2, 4.3),
// built level by level on the device.
//
// The paper's GPU builder recurses on the host and launches two reductions
// per candidate plane.  Here the occupancy of any box of bricks is an O(1)
// query into a 3-D inclusive prefix count over the brick flags (the summed-
// volume-table idea of Sec. 3.2, applied at brick granularity), so a tight
// box is 6 binary searches and one wave evaluates every candidate plane of a
// node at once: lanes take (candidate, side, face) tasks.  Nodes at most 32
// bricks wide read the grid bitmask into occupancy projections instead, from
// which every child box is a few mask operations.  One launch evaluates a
// whole level; its last workgroup to finish numbers the children in
// breadth-first order (left child first) with a block scan.
#include <algorithm>

#include "esk_internal.hpp"
#include "device_util.hpp"

namespace esk {
namespace {

// The k-d build runs beside the renders of the other structures, whose
// waves fill every SIMD; its latency-bound waves raise their issue priority
// so that each level's chain of dependent steps is not slowed to a share of
// its SIMD (the renders lose little: they wait on memory most cycles).
__device__ inline void kd_priority() { __builtin_amdgcn_s_setprio(3); }

// ---------------------------------------------------------------------------
// 3-D inclusive prefix count S over the flags (one pass per axis)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_prefix_axis(KdArgs k, int axis)
{
    kd_priority();
    const int64_t nbx = k.nb[0], nby = k.nb[1], nbz = k.nb[2];
    const int64_t line = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t base, stride, len;
    if (axis == 0) {          // lines along x, indexed by (y, z)
        if (line >= nby * nbz) return;
        base = line * nbx; stride = 1; len = nbx;
    } else if (axis == 1) {   // along y, indexed by (x, z)
        if (line >= nbx * nbz) return;
        const int64_t x = line % nbx, z = line / nbx;
        base = x + nbx * nby * z; stride = nbx; len = nby;
    } else {                  // along z, indexed by (x, y)
        if (line >= nbx * nby) return;
        base = line; stride = nbx * nby; len = nbz;
    }
    int32_t run = 0;
    for (int64_t i = 0; i < len; ++i) {
        const int64_t idx = base + i * stride;
        run += (axis == 0) ? (int32_t)k.flags[idx] : k.S[idx];
        k.S[idx] = run;
    }
}

struct Box {
    int lo[3], hi[3];
};

// S: inclusive prefix count (global memory or an LDS copy), nbx x nby x nbz
template <typename SP>
__device__ inline int32_t S_at(const KdArgs &k, SP S, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0) return 0;
    return S[x + k.nb[0] * (y + k.nb[1] * z)];
}

// number of flagged bricks in [lo, hi)
template <typename SP>
__device__ inline int32_t box_count(const KdArgs &k, SP S, const int lo[3], const int hi[3])
{
    if (hi[0] <= lo[0] || hi[1] <= lo[1] || hi[2] <= lo[2]) return 0;
    const int x0 = lo[0] - 1, y0 = lo[1] - 1, z0 = lo[2] - 1;
    const int x1 = hi[0] - 1, y1 = hi[1] - 1, z1 = hi[2] - 1;
    return S_at(k, S, x1, y1, z1) - S_at(k, S, x0, y1, z1) - S_at(k, S, x1, y0, z1) -
           S_at(k, S, x1, y1, z0) + S_at(k, S, x0, y0, z1) + S_at(k, S, x0, y1, z0) +
           S_at(k, S, x1, y0, z0) - S_at(k, S, x0, y0, z0);
}

// one face of the tight box of region [lo, hi) (which must hold a flagged
// brick): face q in 0..2 = lower bound on axis q, 3..5 = upper bound (exclusive)
template <typename SP>
__device__ inline int tight_face(const KdArgs &k, SP S, const int lo[3], const int hi[3], int face)
{
    const int q = face % 3;
    int a = lo[q], b = hi[q] - 1;
    int l[3] = {lo[0], lo[1], lo[2]}, h[3] = {hi[0], hi[1], hi[2]};
    if (face < 3) {            // smallest c with a flagged brick in [lo_q, c]
        while (a < b) {
            const int m = (a + b) >> 1;
            h[q] = m + 1;
            if (box_count(k, S, l, h) > 0) b = m; else a = m + 1;
        }
        return a;
    }
    while (a < b) {            // largest c with a flagged brick in [c, hi_q)
        const int m = (a + b + 1) >> 1;
        l[q] = m;
        if (box_count(k, S, l, h) > 0) a = m; else b = m - 1;
    }
    return a + 1;
}

__device__ inline int64_t box_volume(const KdArgs &k, const int lo[3], const int hi[3])
{
    int64_t v = 1;
    for (int q = 0; q < 3; ++q) v *= (int64_t)min(k.B * hi[q], k.n[q]) - (int64_t)k.B * lo[q];
    return v;
}

// root: tight box of all flagged bricks (6 lanes of one wave)
__global__ __launch_bounds__(64) void k_kd_root(KdArgs k)
{
    kd_priority();
    __shared__ int face[6];
    const int lane = threadIdx.x;
    const int lo[3] = {0, 0, 0}, hi[3] = {k.nb[0], k.nb[1], k.nb[2]};
    const int32_t total = box_count(k, (const int32_t *)k.S, lo, hi);
    if (total == 0) {
        if (lane == 0) {
            k.hdr->kd_count = 0;
            k.hdr->kd_height = 0;
            k.hdr->kd_begin = 0;
            k.hdr->kd_end = 0;
            k.hdr->kd_ticket = 0;
            k.hdr->pad[0] = 0;
            k.hdr->kd_next[0][0] = kKdNumbered;
            k.hdr->kd_next[0][1] = 0;
            k.hdr->kd_next[0][2] = 0;
        }
        return;
    }
    if (lane < 6) face[lane] = tight_face(k, (const int32_t *)k.S, lo, hi, lane);
    __syncthreads();
    if (lane < 3) {
        k.lo[lane] = face[lane];
        k.hi[lane] = face[3 + lane];
    }
    if (lane == 0) {
        k.hdr->kd_count = 1;
        k.hdr->kd_height = 1;
        k.hdr->kd_begin = 0;
        k.hdr->kd_end = 1;
        k.hdr->kd_ticket = 0;
        k.hdr->pad[0] = 0;
        k.hdr->kd_next[0][0] = kKdNumbered;
        k.hdr->kd_next[0][1] = 0;
        k.hdr->kd_next[0][2] = 1;
    }
}

// the j-th candidate plane of node box [lo, hi): planes lo + floor(i*e/bins),
// i = 1..bins-1, inside (lo, hi), deduplicated, axes in order x, y, z.
// Returns the count; fills (axis, plane) for index `want` if it exists.
__device__ inline int candidate(const int lo[3], const int hi[3], int bins, int want, int *ax, int *pl)
{
    int c = 0;
    for (int a = 0; a < 3; ++a) {
        const int e = hi[a] - lo[a];
        if (e < 2) continue;
        int prev = -1;
        for (int j = 1; j < bins; ++j) {
            const int p = lo[a] + (int)(((int64_t)j * e) / bins);
            if (p <= lo[a] || p >= hi[a] || p == prev) continue;
            prev = p;
            if (c == want) { *ax = a; *pl = p; }
            ++c;
        }
    }
    return c;
}

constexpr int kMaxCand = 45;   // 3 axes x (16 bins - 1)

// Boxes up to this many bricks along every axis read their projections entry
// by entry (a few entries: cheaper than building the tables below).
constexpr int kProjLoopMax = 8;

// Occupancy projections of a node whose brick box is at most 32 bricks along
// every axis, relative to the box: X[y] = the x-bitmask of the flagged bricks
// of row y (any z), XZ[z] = the x-bitmask of slab z (any y), YZ[z] = the
// y-bitmask of slab z (bit y set where row (y, z) holds a flagged brick),
// and their transposes Tyx[x] (the rows holding column x), Tzx[x] (the
// slabs holding column x) and Tzy[y] (the slabs holding row y).  Every
// child box of a candidate plane is then a union over a prefix or a suffix
// of one of these arrays (below), so the wave keeps, per array, the unions
// of every prefix and every suffix: each (candidate, side) task is three
// table reads instead of six binary searches over the prefix count (each
// step a dependent round of eight loads) or a loop over the 32 entries.
struct __align__(16) Proj {
    uint32_t X[32], XZ[32], YZ[32];
    union {
        uint32_t T[32][33];   // T[z][y]: the x-bitmask of row (y, z) (padded: conflict-free columns)
        uint32_t tab[64][8];  // afterwards: per lane, the prefix / suffix unions (see build_proj)
    };
    int16_t ca[kMaxCand], cp[kMaxCand];   // the node's candidate planes: axis, plane
};

__device__ inline uint32_t low_bits(int n) { return n >= 32 ? 0xffffffffu : ((1u << n) - 1u); }

// Transpose of the bit matrix held by each half of the wave (lane r of the
// half holds row r, bit c its column c), nonzero only in its first `span`
// rows and columns (a power of two): afterwards lane c holds column c.
// Rounds of swapping the off-diagonal blocks of halving size; the blocks of
// the rounds skipped (size >= span) are zero.
__device__ inline uint32_t transpose32(uint32_t v, int span)
{
    const int lane = threadIdx.x & 63;
    constexpr uint32_t keep[5] = {0x0000ffffu, 0x00ff00ffu, 0x0f0f0f0fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int j = 16 >> s;
        if (j >= span) continue;   // wave-uniform
        const uint32_t m = keep[s];
        const uint32_t o = (uint32_t)__shfl_xor((int)v, j, 64);
        v = (lane & j) ? ((v & ~m) | ((o & ~m) >> j)) : ((v & m) | ((o & m) << j));
    }
    return v;
}

// unions over the lanes before (exclusive) and from (inclusive) each lane of
// its 32-lane half, for the lanes below `span` (entries from span on are zero)
__device__ inline void or_scans(uint32_t v, int span, uint32_t &pre, uint32_t &suf)
{
    uint32_t a = v, b = v;
    for (int d = 1; d < span; d <<= 1) {
        a |= (uint32_t)__shfl_up((int)a, d, 32);
        b |= (uint32_t)__shfl_down((int)b, d, 32);
    }
    // every lane takes part in the shuffle (a lane outside EXEC supplies zero), then selects
    const uint32_t prev = (uint32_t)__shfl_up((int)a, 1, 32);
    pre = (threadIdx.x & 31) == 0 ? 0u : prev;
    suf = b;
}

// One wave.  Lane (y, h) reads the rows (y, z) with z of parity h from the
// grid bitmask, 16 slabs' words in flight per round; X accumulates in
// registers, YZ is a ballot per slab, XZ an OR over the rows of the slab.
// Then per half of the wave r1 = X (lanes 0-31) | XZ (lanes 32-63), r2 = YZ
// (lanes 0-31), their transposes t1 = Tyx | Tzx and t2 = Tzy, and tab[lane]
// = {pre r1, suf r1, pre r2, suf r2, pre t1, suf t1, pre t2, suf t2}.
// Entries past the box's extents are zero.
// The row reads of build_proj: P->T[z][y] = the x-bitmask of row (y, z) of
// the box, P->YZ[z] = the y-bitmask of its non-empty rows; returns the OR of
// the lane's rows (lane (y, h): rows (y, z), z of parity h).
__device__ inline uint32_t proj_rows(const KdArgs &k, const int lo[3], const int hi[3], Proj *P)
{
    const int lane = threadIdx.x & 63;
    const int y = lane & 31, h = lane >> 5;
    const int ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    const uint32_t full = low_bits(ex);
    const uint64_t nb0 = (uint64_t)k.nb[0], nb1 = (uint64_t)k.nb[1];
    uint32_t xacc = 0u;
    // rounds of 16 slabs, each row's words in flight before the first is used
    for (int z0 = 0; z0 < ez; z0 += 16) {
        uint32_t lw[8], hw[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            lw[u] = 0u;
            hw[u] = 0u;
            if (z0 + 2 * u >= ez) continue;   // wave-uniform
            const int z = z0 + 2 * u + h;
            if (y < ey && z < ez) {
                // bits [base, base + ex) of the bitmask: the row's bricks lo_x .. hi_x - 1
                const uint64_t base =
                    nb0 * ((uint64_t)(lo[1] + y) + nb1 * (uint64_t)(lo[2] + z)) + (uint64_t)lo[0];
                const uint64_t wi = base >> 5;
                lw[u] = k.grid[wi];
                if ((int)(base & 31u) + ex > 32) hw[u] = k.grid[wi + 1];   // the row's last brick lies there
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (z0 + 2 * u >= ez) continue;   // wave-uniform
            const int z = z0 + 2 * u + h;
            const bool in = y < ey && z < ez;
            const uint64_t base = nb0 * ((uint64_t)(lo[1] + y) + nb1 * (uint64_t)(lo[2] + z)) + (uint64_t)lo[0];
            const uint64_t w = (uint64_t)lw[u] | ((uint64_t)hw[u] << 32);
            const uint32_t m = in ? (uint32_t)(w >> (int)(base & 31u)) & full : 0u;
            xacc |= m;
            const uint64_t bal = __ballot(m != 0u);
            if (z < ez) {
                P->T[z][y] = m;
                if (y == 0) P->YZ[z] = (uint32_t)(bal >> (32 * h));
            }
        }
    }
    wave_lds_sync();
    return xacc;
}

__device__ inline void build_proj(const KdArgs &k, const int lo[3], const int hi[3], Proj *P)
{
    const int lane = threadIdx.x & 63;
    const int y = lane & 31, h = lane >> 5;
    const int ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    const uint32_t xacc = proj_rows(k, lo, hi, P);
    const uint32_t xo = xacc | (uint32_t)__shfl_xor((int)xacc, 32, 64);   // even and odd slabs
    uint32_t xz = 0u;
    if (h == 1 && y < ez) {
#pragma unroll 8
        for (int yy = 0; yy < ey; ++yy) xz |= P->T[y][yy];
    }
    const int n = max(ex, max(ey, ez));
    if (n <= kProjLoopMax) {
        // the entries themselves (zero past the extents, but YZ)
        if (h == 0) P->X[y] = xo; else P->XZ[y] = xz;
        wave_lds_sync();
        return;
    }
    const uint32_t r1 = h == 0 ? xo : xz;
    const uint32_t r2 = h == 0 && y < ez ? P->YZ[y] : 0u;
    wave_lds_sync();   // T is overwritten by the tables
    // the smallest power of two covering every extent: the arrays are zero from there on
    const int span = n <= 1 ? 1 : 1 << (32 - __builtin_clz((uint32_t)(n - 1)));
    const uint32_t t1 = transpose32(r1, span), t2 = transpose32(r2, span);
    uint4 lo4, hi4;
    or_scans(r1, span, lo4.x, lo4.y);
    or_scans(r2, span, lo4.z, lo4.w);
    or_scans(t1, span, hi4.x, hi4.y);
    or_scans(t2, span, hi4.z, hi4.w);
    uint4 *row = reinterpret_cast<uint4 *>(P->tab[lane]);
    row[0] = lo4;
    row[1] = hi4;
    wave_lds_sync();
}

// The candidate planes of box [lo, hi) in order (axes x, y, z; planes
// lo + floor(i e / bins), i = 1 .. bins - 1, strictly inside, a plane equal
// to the one before it on its axis dropped), one per lane, compacted into
// P->ca / P->cp; returns their count.  The same list as candidate().
__device__ inline int candidates_lds(const int lo[3], const int hi[3], int bins, Proj *P)
{
    const int lane = threadIdx.x & 63;
    const int per = bins - 1;
    bool ok = false;
    int a = 0, p = 0;
    if (lane < 3 * per) {
        a = lane / per;
        const int i = lane % per + 1;
        const int e = hi[a] - lo[a];
        p = lo[a] + (i * e) / bins;
        const int prev = i > 1 ? lo[a] + ((i - 1) * e) / bins : -1;
        ok = e >= 2 && p > lo[a] && p < hi[a] && p != prev;
    }
    const uint64_t bal = __ballot(ok);
    if (ok) {
        const int rank = __popcll(bal & ((1ull << lane) - 1ull));
        P->ca[rank] = (int16_t)a;
        P->cp[rank] = (int16_t)p;
    }
    wave_lds_sync();
    return __popcll(bal);
}

// The x-, y- and z-bitmasks (relative to the box) of the node's bricks below
// (side 0) or at and above (side 1) plane p on axis a, from the entries: one
// loop over them for every axis, with selects (lanes of a wave take
// different axes), the entries read four at a time.
__device__ inline void proj_masks_loop(const Proj *P, const int lo[3], const int hi[3], int a, int p, int side,
                                       uint32_t m[3])
{
    const int ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    const int ea = hi[a] - lo[a];
    const uint32_t below = low_bits(p - lo[a]);
    const uint32_t am = side == 0 ? below : (low_bits(ea) & ~below);
    const bool ax = a == 0, ay = a == 1;
    const int n = max(ey, ez);
    uint32_t mx = 0u, my = 0u, mz = 0u;
    const uint4 *X4 = reinterpret_cast<const uint4 *>(P->X);
    const uint4 *XZ4 = reinterpret_cast<const uint4 *>(P->XZ);
    const uint4 *YZ4 = reinterpret_cast<const uint4 *>(P->YZ);
    for (int i0 = 0; i0 < n; i0 += 4) {
        const uint4 xq = X4[i0 >> 2], xzq = XZ4[i0 >> 2], yzq = YZ4[i0 >> 2];
        const uint32_t xv[4] = {xq.x, xq.y, xq.z, xq.w};
        const uint32_t xzv[4] = {xzq.x, xzq.y, xzq.z, xzq.w};
        const uint32_t yzv[4] = {yzq.x, yzq.y, yzq.z, yzq.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u;
            const uint32_t bit = 1u << (i & 31);
            // YZ entries past the box's extent hold an earlier node's values
            const uint32_t X = i < ey ? xv[u] : 0u;
            const uint32_t XZ = i < ez ? xzv[u] : 0u;
            const uint32_t YZ = i < ez ? yzv[u] : 0u;
            const bool in = ((am >> (i & 31)) & 1u) != 0u;
            // split along x: i is y for X, z for XZ
            const uint32_t qx = X & am;
            // split along y: i is y for X, z for YZ
            const uint32_t qy = YZ & am;
            mx |= ax ? qx : (ay ? (in ? X : 0u) : (in ? XZ : 0u));
            my |= ax ? (qx ? bit : 0u) : (ay ? qy : (in ? YZ : 0u));
            mz |= ax ? ((XZ & am) ? bit : 0u) : (ay ? (qy ? bit : 0u) : ((in && YZ) ? bit : 0u));
        }
    }
    m[0] = mx;
    m[1] = my;
    m[2] = mz;
}

// The same bitmasks from the tables.  With q = p - lo[a] and side 0 taking
// entries [0, q), side 1 entries [q, extent):
//   a = x: x-bits = X(all) & side, y-bits = union of Tyx, z-bits = union of Tzx
//   a = y: x-bits = union of X,  y-bits = Y(all) & side, z-bits = union of Tzy
//   a = z: x-bits = union of XZ, y-bits = union of YZ, z-bits = Z(all) & side
// where the unions run over the side's entries (a prefix or a suffix).
__device__ inline void proj_masks_tab(const Proj *P, const int lo[3], const int hi[3], int a, int p, int side,
                                      uint32_t m[3])
{
    const int q = p - lo[a];
    const uint32_t below = low_bits(q);
    const uint32_t am = side == 0 ? below : (low_bits(hi[a] - lo[a]) & ~below);
    const uint32_t *t = &P->tab[0][0];
    // tab[lane][2 * array + side], arrays r1, r2, t1, t2 (build_proj)
    const uint32_t vx = t[(a == 2 ? 32 + q : q) * 8 + side];
    const uint32_t vy = t[q * 8 + (a == 0 ? 4 : 2) + side];
    const uint32_t vz = t[(a == 0 ? 32 + q : q) * 8 + (a == 0 ? 4 : 6) + side];
    // the unions of whole arrays: X over all rows, Y = rows holding a brick (YZ over all
    // slabs), Z = slabs holding a brick (Tzx over all columns)
    m[0] = a == 0 ? (t[0 * 8 + 1] & am) : vx;
    m[1] = a == 1 ? (t[0 * 8 + 3] & am) : vy;
    m[2] = a == 2 ? (t[32 * 8 + 5] & am) : vz;
}

// faces (absolute brick coordinates: lower bounds, then exclusive upper
// bounds) of the tight box of the node's bricks below (side 0) or at and
// above (side 1) plane p on axis a; both sides of a plane strictly inside a
// tight box hold a flagged brick.
__device__ inline void proj_child(const Proj *P, const int lo[3], const int hi[3], int a, int p, int side, int f[6])
{
    const int n = max(hi[0] - lo[0], max(hi[1] - lo[1], hi[2] - lo[2]));
    uint32_t m[3];
    if (n <= kProjLoopMax)   // wave-uniform: the node's box
        proj_masks_loop(P, lo, hi, a, p, side, m);
    else
        proj_masks_tab(P, lo, hi, a, p, side, m);
    for (int i = 0; i < 3; ++i) {
        f[i] = lo[i] + (int)__builtin_ctz(m[i]);
        f[3 + i] = lo[i] + 32 - (int)__builtin_clz(m[i]);
    }
}

// Decides the split of one node (one wave): the children's tight boxes come
// from the node's occupancy projections where the node spans at most 32
// bricks per axis, else every (candidate plane, side, face) binary search
// over the prefix count runs on its own lane; lane 0 writes axis, plane,
// split flag and the two children's tight boxes, and every lane returns the
// split flag.  plist: the level's
// splitting parents in order (the parent of node begin + r is plist[r / 2]);
// tb, P: this wave's scratch.
template <typename SP>
__device__ bool eval_node(const KdArgs &k, SP S, const int32_t *plist, int64_t node, int64_t begin, int64_t vroot,
                          int16_t (*tb)[2][6], Proj *P)
{
    const int lane = threadIdx.x & 63;
    int lo[3], hi[3];
    if (node == 0) {
        for (int q = 0; q < 3; ++q) {
            lo[q] = k.lo[q];
            hi[q] = k.hi[q];
        }
    } else {
        // child `side` of the (r/2)-th splitting node of the level above: its
        // box from the parent's child boxes, recorded for later readers
        const int64_t r = node - begin;
        const int64_t p = plist[r >> 1];
        const int32_t *cb = &k.clo[12 * p + 6 * (r & 1)];
        for (int q = 0; q < 3; ++q) {
            lo[q] = cb[q];
            hi[q] = cb[3 + q];
        }
        if (lane == 0)
            for (int q = 0; q < 3; ++q) {
                k.lo[3 * node + q] = lo[q];
                k.hi[3 * node + q] = hi[q];
            }
    }
    const int64_t V = box_volume(k, lo, hi);
    const bool allowed = k.halting == 0 ? (10 * V > vroot) : (V > 512);
    // wave-uniform: the box is the same on every lane
    const bool proj = hi[0] - lo[0] <= 32 && hi[1] - lo[1] <= 32 && hi[2] - lo[2] <= 32;
    const int ncand = allowed ? candidates_lds(lo, hi, k.bins, P) : 0;
    if (proj && ncand > 0) build_proj(k, lo, hi, P);
    int best = -1;
    int64_t best_cost = 0;
    if (ncand > 0) {
        if (proj) {
            for (int t = lane; t < ncand * 2; t += 64) {
                const int c = t >> 1, side = t & 1;
                int f[6];
                proj_child(P, lo, hi, P->ca[c], P->cp[c], side, f);
                for (int q = 0; q < 6; ++q) tb[c][side][q] = (int16_t)f[q];
            }
        } else {
            for (int t = lane; t < ncand * 12; t += 64) {
                const int c = t / 12, side = (t / 6) & 1, face = t % 6;
                const int a = P->ca[c], p = P->cp[c];
                int rl[3] = {lo[0], lo[1], lo[2]}, rh[3] = {hi[0], hi[1], hi[2]};
                if (side == 0) rh[a] = p; else rl[a] = p;
                tb[c][side][face] = (int16_t)tight_face(k, S, rl, rh, face);
            }
        }
        wave_lds_sync();
        int64_t cost = 0x7fffffffffffffffLL;
        if (lane < ncand) {
            int L[6], R[6];
            for (int f = 0; f < 6; ++f) { L[f] = tb[lane][0][f]; R[f] = tb[lane][1][f]; }
            cost = box_volume(k, L, L + 3) + box_volume(k, R, R + 3);
        }
        // argmin over (cost, candidate index): lower index wins ties
        int idx = lane < ncand ? lane : 0x7fffffff;
        for (int o = 32; o >= 1; o >>= 1) {
            const int64_t oc = __shfl_xor(cost, o, 64);
            const int oi = __shfl_xor(idx, o, 64);
            if (oc < cost || (oc == cost && oi < idx)) { cost = oc; idx = oi; }
        }
        best = idx;
        best_cost = cost;
    }
    int axis = -1, plane = 0;
    int cl[2][6];
    if (best >= 0 && best_cost < V) {
        axis = P->ca[best];
        plane = P->cp[best];
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 6; ++f) cl[s][f] = tb[best][s][f];
    } else if (best >= 0 && k.max_leaf > 0 &&
               V > (int64_t)k.max_leaf * k.max_leaf * k.max_leaf) {
        // maximum leaf size: middle of the axis with the largest voxel extent
        int64_t best_ext = -1;
        for (int a = 0; a < 3; ++a) {
            const int e = hi[a] - lo[a];
            if (e < 2) continue;
            const int64_t ext = (int64_t)min(k.B * hi[a], k.n[a]) - (int64_t)k.B * lo[a];
            if (ext > best_ext) { best_ext = ext; axis = a; plane = lo[a] + e / 2; }
        }
        wave_lds_sync();
        if (proj) {
            if (lane < 2) {
                int f[6];
                proj_child(P, lo, hi, axis, plane, lane, f);
                for (int q = 0; q < 6; ++q) tb[kMaxCand][lane][q] = (int16_t)f[q];
            }
        } else if (lane < 12) {
            const int side = lane / 6, face = lane % 6;
            int rl[3] = {lo[0], lo[1], lo[2]}, rh[3] = {hi[0], hi[1], hi[2]};
            if (side == 0) rh[axis] = plane; else rl[axis] = plane;
            tb[kMaxCand][side][face] = (int16_t)tight_face(k, S, rl, rh, face);
        }
        wave_lds_sync();
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 6; ++f) cl[s][f] = tb[kMaxCand][s][f];
    }
    if (lane == 0) {
        k.axis[node] = axis;
        k.plane[node] = axis >= 0 ? plane : 0;
        k.split[node] = axis >= 0 ? 1 : 0;
        if (axis >= 0)
            for (int s = 0; s < 2; ++s)
                for (int f = 0; f < 6; ++f) k.clo[12 * node + 6 * s + f] = cl[s][f];
        if (axis < 0) k.first[node] = -1;
    }
    wave_lds_sync();
    return axis >= 0;   // wave-uniform
}

__device__ inline int64_t root_volume(const KdArgs &k)
{
    const int rlo[3] = {k.lo[0], k.lo[1], k.lo[2]}, rhi[3] = {k.hi[0], k.hi[1], k.hi[2]};
    return box_volume(k, rlo, rhi);
}

// Grids of at most 32 bricks along every axis, brick-granular cost: every
// node spans at most 32 bricks, so every node is evaluated from occupancy
// projections and the prefix count is never read.  The root's tight box then
// comes from the projections of the whole grid (one wave): the x-bits of
// every row, the rows and the slabs holding a flagged brick.
__global__ __launch_bounds__(64) void k_kd_root_bits(KdArgs k)
{
    kd_priority();
    __shared__ Proj P;
    const int lane = threadIdx.x;
    const int lo[3] = {0, 0, 0}, hi[3] = {k.nb[0], k.nb[1], k.nb[2]};
    uint32_t xall = proj_rows(k, lo, hi, &P);
    const uint32_t yz = lane < hi[2] ? P.YZ[lane] : 0u;
    uint32_t yall = yz;
    for (int o = 32; o >= 1; o >>= 1) {
        xall |= (uint32_t)__shfl_xor((int)xall, o, 64);
        yall |= (uint32_t)__shfl_xor((int)yall, o, 64);
    }
    const uint32_t zall = (uint32_t)__ballot(yz != 0u);
    if (lane == 0) {
        const bool any = xall != 0u;
        if (any) {
            const uint32_t m[3] = {xall, yall, zall};
            for (int a = 0; a < 3; ++a) {
                k.lo[a] = (int)__builtin_ctz(m[a]);
                k.hi[a] = 32 - (int)__builtin_clz(m[a]);
            }
        }
        k.hdr->kd_count = any ? 1u : 0u;
        k.hdr->kd_height = any ? 1u : 0u;
        k.hdr->kd_begin = 0;
        k.hdr->kd_end = any ? 1u : 0u;
        k.hdr->kd_ticket = 0;
        k.hdr->pad[0] = 0;
        k.hdr->kd_next[0][0] = kKdNumbered;
        k.hdr->kd_next[0][1] = 0;
        k.hdr->kd_next[0][2] = any ? 1u : 0u;
    }
}

// Small grids (<= 32768 bricks): the 3-D prefix count is built in LDS by one
// workgroup, written out, and the root's tight box found -- one launch
// instead of three prefix passes plus the root kernel.
constexpr int kKdSmallBricks = 32768;

__global__ __launch_bounds__(1024) void k_kd_prefix_root_small(KdArgs k)
{
    kd_priority();
    extern __shared__ int32_t S[];
    const int nbx = k.nb[0], nby = k.nb[1], nbz = k.nb[2];
    const int nb = nbx * nby * nbz;
    const int t = threadIdx.x;
    for (int line = t; line < nby * nbz; line += 1024) {
        int run = 0;
        for (int x = 0; x < nbx; ++x) {
            run += k.flags[(int64_t)line * nbx + x];
            S[line * nbx + x] = run;
        }
    }
    __syncthreads();
    for (int line = t; line < nbx * nbz; line += 1024) {
        const int x = line % nbx, z = line / nbx;
        int run = 0;
        for (int y = 0; y < nby; ++y) {
            const int idx = x + nbx * (y + nby * z);
            run += S[idx];
            S[idx] = run;
        }
    }
    __syncthreads();
    for (int line = t; line < nbx * nby; line += 1024) {
        int run = 0;
        for (int z = 0; z < nbz; ++z) {
            const int idx = line + nbx * nby * z;
            run += S[idx];
            S[idx] = run;
        }
    }
    __syncthreads();
    for (int i = t; i < nb; i += 1024) k.S[i] = S[i];
    const int glo[3] = {0, 0, 0}, ghi[3] = {nbx, nby, nbz};
    const bool any = box_count(k, (const int32_t *)S, glo, ghi) > 0;
    if (any && t < 6) {
        const int f = tight_face(k, (const int32_t *)S, glo, ghi, t);
        if (t < 3) k.lo[t] = f; else k.hi[t - 3] = f;
    }
    if (t == 0) {
        k.hdr->kd_count = any ? 1u : 0u;
        k.hdr->kd_height = any ? 1u : 0u;
        k.hdr->kd_begin = 0;
        k.hdr->kd_end = any ? 1u : 0u;
        k.hdr->kd_ticket = 0;
        k.hdr->pad[0] = 0;
        k.hdr->kd_next[0][0] = kKdNumbered;
        k.hdr->kd_next[0][1] = 0;
        k.hdr->kd_next[0][2] = any ? 1u : 0u;
    }
}

// The first levels of a tree, while they hold at most kKdTopWaves nodes,
// in one workgroup: a wave per node, the children numbered in LDS by one
// thread between levels (workgroup barriers instead of launches).  It hands
// the first wider level over to the level launches as a numbered level (its
// parents in the global list, slot 0) and records how many levels it took.
constexpr int kKdTopWaves = 8;

__global__ __launch_bounds__(64 * kKdTopWaves) void k_kd_top(KdArgs k)
{
    kd_priority();
    __shared__ int16_t tb[kKdTopWaves][kMaxCand + 1][2][6];
    __shared__ Proj proj[kKdTopWaves];
    __shared__ int32_t parents[kKdTopWaves];
    __shared__ int32_t split[kKdTopWaves];
    __shared__ uint32_t level[3];   // begin, end, levels taken
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        level[0] = k.hdr->kd_next[0][1];
        level[1] = k.hdr->kd_next[0][2];
        level[2] = 0;
    }
    __syncthreads();
    const int64_t vroot = root_volume(k);
    uint32_t height = k.hdr->kd_height;
    while (true) {
        const uint32_t begin = level[0], end = level[1];
        if (end == begin || end - begin > (uint32_t)kKdTopWaves) break;
        const int64_t node = (int64_t)begin + wave;
        bool sp = false;
        if (node < end)
            sp = eval_node(k, (const int32_t *)k.S, level[2] == 0 ? k.plist : parents, node, (int64_t)begin, vroot,
                           tb[wave], &proj[wave]);
        if (node < end && lane == 0) split[wave] = sp ? 1 : 0;
        __syncthreads();   // also makes the waves' global stores (child boxes) visible to the block
        if (threadIdx.x == 0) {
            uint32_t total = 0;
            for (uint32_t i = 0; i < end - begin; ++i) total += split[i] ? 1u : 0u;
            const bool fits = (int64_t)end + 2 * (int64_t)total <= k.cap;
            uint32_t run = 0;
            if (fits)
                for (uint32_t i = 0; i < end - begin; ++i)
                    if (split[i]) {
                        parents[run] = (int32_t)(begin + i);
                        k.plist[run] = (int32_t)(begin + i);
                        k.first[begin + i] = (int32_t)((int64_t)end + 2 * (int64_t)run);
                        ++run;
                    }
            if (!fits) k.hdr->pad[0] = 1u;  // cannot happen for a correct build: stop growing
            level[0] = end;
            level[1] = fits ? end + 2 * total : end;
            level[2] += 1;
        }
        __syncthreads();
        if (level[1] > level[0]) height += 1;
    }
    if (threadIdx.x == 0) {
        const uint32_t begin = level[0], end = level[1];
        k.hdr->kd_begin = begin;
        k.hdr->kd_end = end;
        k.hdr->kd_count = end;
        k.hdr->kd_height = height;
        k.hdr->kd_top_levels = level[2];
        k.hdr->kd_next[0][0] = kKdNumbered;
        k.hdr->kd_next[0][1] = begin;
        k.hdr->kd_next[0][2] = end;
    }
}

// One level per launch, no host round trip: the level bounds come from the
// device header (a level past the last one finds begin == end and exits).
// Waves of a fixed grid evaluate the level's nodes.  The children of a level
// of at most kKdNumberLds nodes are numbered by every block of the next
// launch from the split flags; those of a wider level by the last block of
// its own launch to finish (ticket counter, agent-scope release/acquire),
// which publishes the next level.  Either way in breadth-first order.
// Workgroups per level launch, from the brick count: nb / 128 up to 256
// (four waves each, so a level of up to 1024 nodes -- the widest levels of
// 32^3 bricks hold ~500 -- is evaluated in one round of its waves instead
// of several rounds of dependent loads), nb / 1024 beyond, clamped to
// [32, 1024].  Measured on 32^3 bricks: 32 blocks 0.33 ms, 128 0.29, 256
// 0.28 ms for the k-d rebuild, the whole step the same within noise.
inline int kd_level_blocks(const KdArgs &k)
{
    const int64_t nb = (int64_t)k.nb[0] * k.nb[1] * k.nb[2];
    const int64_t want = std::max<int64_t>(std::min<int64_t>(256, nb / 128), nb / 1024);
    return (int)std::min<int64_t>(1024, std::max<int64_t>(32, want));
}

// Breadth-first numbering of the children of level [begin, end) by one
// 256-thread workgroup, the last of the level's launch to finish (every
// split flag of the level is visible to it): children in parent order, the
// first child of each splitting parent, the ordered list of splitting
// parents, and the next level's bounds in the header.
__device__ void number_children(const KdArgs &k, uint32_t begin, uint32_t end, uint32_t *scratch, uint32_t *slot)
{
    const int64_t width = (int64_t)end - begin;
    const int64_t per = (width + 255) / 256;
    const int64_t i0 = begin + threadIdx.x * per;
    const int64_t i1 = min((int64_t)end, i0 + per);
    // plain loads of the flags (the caller's acquire made them visible),
    // eight at a time so the loads overlap instead of waiting one by one
    constexpr int U = 8;
    uint32_t c = 0;
    {
        int64_t i = i0;
        for (; i + U <= i1; i += U) {
            int32_t f[U];
#pragma unroll
            for (int u = 0; u < U; ++u) f[u] = k.split[i + u];
#pragma unroll
            for (int u = 0; u < U; ++u) c += f[u] != 0 ? 1u : 0u;
        }
        for (; i < i1; ++i) c += k.split[i] != 0 ? 1u : 0u;
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<256>(c, scratch, &total);
    const bool fits = (int64_t)end + 2 * (int64_t)total <= k.cap;
    if (fits) {
        // children are numbered in parent order; each child reads its box
        // from the parent's record when its own level is evaluated
        const int32_t *__restrict__ sp = k.split;
        int32_t *__restrict__ fp = k.first;
        int32_t *__restrict__ pl = k.plist;
        int64_t i = i0;
        for (; i + U <= i1; i += U) {
            int32_t f[U];
#pragma unroll
            for (int u = 0; u < U; ++u) f[u] = sp[i + u];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (f[u]) {
                    fp[i + u] = (int32_t)((int64_t)end + 2 * (int64_t)run);
                    pl[run] = (int32_t)(i + u);
                    ++run;
                }
        }
        for (; i < i1; ++i)
            if (sp[i]) {
                fp[i] = (int32_t)((int64_t)end + 2 * (int64_t)run);
                pl[run] = (int32_t)i;
                ++run;
            }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!fits) k.hdr->pad[0] = 1u;  // cannot happen for a correct build: stop growing
        const uint32_t next = fits ? end + 2 * total : end;
        k.hdr->kd_begin = end;
        k.hdr->kd_end = next;
        k.hdr->kd_count = next;
        if (fits && total > 0) k.hdr->kd_height += 1;
        k.hdr->kd_ticket = 0;
        if (slot) {
            slot[0] = kKdNumbered;
            slot[1] = end;
            slot[2] = next;
        }
        __threadfence();
    }
}

// Widest level whose children the next level launch numbers itself: every
// block of that launch scans the level's split flags (at most 8 per thread)
// and lists the splitting parents in LDS, so no block of the level's own
// launch waits for the others (no ticket, no last-block numbering).
constexpr int kKdNumberLds = 2048;

// Numbering of the children of the level [pb, pe) (pe - pb <= kKdNumberLds),
// done by every block of the launch that evaluates them: the splitting
// parents in order into parents[], the children's level into [*begin, *end).
// Block 0 also records each splitting parent's first child and the level in
// the header, as number_children does.
__device__ void number_in_block(const KdArgs &k, uint32_t pb, uint32_t pe, int32_t *parents, uint32_t *scratch,
                                uint32_t *begin, uint32_t *end)
{
    constexpr int U = kKdNumberLds / 256;
    const int64_t width = (int64_t)pe - pb;
    const int64_t per = (width + 255) / 256;   // <= U
    const int64_t i0 = pb + threadIdx.x * per;
    const int64_t i1 = min((int64_t)pe, i0 + per);
    int32_t f[U];
    uint32_t c = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        f[u] = i0 + u < i1 ? k.split[i0 + u] : 0;
        c += f[u] != 0 ? 1u : 0u;
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<256>(c, scratch, &total);
    const bool fits = (int64_t)pe + 2 * (int64_t)total <= k.cap;
    const bool first = blockIdx.x == 0 && fits;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (f[u]) {
            parents[run] = (int32_t)(i0 + u);
            if (first) k.first[i0 + u] = (int32_t)((int64_t)pe + 2 * (int64_t)run);
            ++run;
        }
    __syncthreads();
    const uint32_t next = fits ? pe + 2 * total : pe;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!fits) k.hdr->pad[0] = 1u;  // cannot happen for a correct build: stop growing
        k.hdr->kd_begin = pe;
        k.hdr->kd_end = next;
        k.hdr->kd_count = next;
        if (fits && total > 0) k.hdr->kd_height += 1;
    }
    *begin = pe;
    *end = next;
}

// The last workgroup of a level launch to arrive (ticket counter) numbers
// the children.  Every wave first waits for its own stores; one agent-scope
// release per workgroup then publishes them (on a multi-XCD part a release
// writes back the XCD's L2, so it is not issued per node).
__device__ inline bool last_of_level(const KdArgs &k, uint32_t *last)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(&k.hdr->kd_ticket, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        *last = (old == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!*last) return false;
    // plain loads of the flags follow: this acquire (agent scope) follows the
    // other blocks' release through the ticket, so their flags are visible
    __threadfence();
    return true;
}

// The binary searches read the prefix count through L2 (staging the whole
// table in LDS per workgroup was measured slower: every busy workgroup of a
// level copies it again).  li: the launch's index in the build (its slot of
// kd_next is li % 2; it writes the other one for the next launch).
__global__ __launch_bounds__(256) void k_kd_level(KdArgs k, uint32_t li)
{
    kd_priority();
    __shared__ int16_t tb[4][kMaxCand + 1][2][6];
    __shared__ Proj proj[4];
    __shared__ uint32_t scratch[5];
    __shared__ uint32_t last;
    __shared__ int32_t parents[kKdNumberLds];
    const uint32_t *in = k.hdr->kd_next[li & 1u];
    uint32_t *out = k.hdr->kd_next[(li + 1u) & 1u];
    const uint32_t mode = in[0];
    uint32_t begin = in[1], end = in[2];
    const int32_t *plist = k.plist;
    if (mode == kKdToNumber) {
        // the launch before evaluated [begin, end) and left its children to this one
        number_in_block(k, begin, end, parents, scratch, &begin, &end);
        plist = parents;
    }
    const uint32_t width = end - begin;
    const bool narrow = width <= (uint32_t)kKdNumberLds;
    if (narrow && blockIdx.x == 0 && threadIdx.x == 0) {
        // the next launch numbers this level's children (or finds the build finished)
        out[0] = width == 0 ? kKdNumbered : kKdToNumber;
        out[1] = begin;
        out[2] = end;
    }
    if (width == 0) return;
    const int wave = threadIdx.x >> 6;
    const int64_t vroot = root_volume(k);
    for (int64_t node = (int64_t)begin + (int64_t)blockIdx.x * 4 + wave; node < end;
         node += (int64_t)gridDim.x * 4) {
        eval_node(k, (const int32_t *)k.S, plist, node, (int64_t)begin, vroot, tb[wave], &proj[wave]);
    }
    // a wide level: the last block to finish numbers the children and fills the next slot
    if (!narrow && last_of_level(k, &last)) number_children(k, begin, end, scratch, out);
}

// ---------------------------------------------------------------------------
// The voxel-tight split cost (Sec. 3.2.2: the GPU builder keeps one tight box
// per macro cell and reduces over the cells of a region).  One workgroup per
// node: the voxel-tight boxes of the flagged bricks in the node's brick box
// are reduced into per-slab unions along each axis (LDS, 6 ints per brick
// slab, atomics), so the union left and right of every candidate plane is a
// prefix / suffix over one axis's slabs.  Every volume the rules compare is
// the half-voxel volume of such a union (0 without a visible cell): a side's
// cost, the node's own (split iff the best cost is below it), the root's
// (shallow halting), 8^3 and MLS^3 voxels (x 8).  Regions, candidate planes,
// the maximum-leaf-size plane and the children (brick-tight, from the prefix
// count) stay on the brick raster.
// ---------------------------------------------------------------------------

__device__ inline int64_t half_volume(const int l[3], const int h[3])
{
    if (h[0] <= l[0] || h[1] <= l[1] || h[2] <= l[2]) return 0;
    return (int64_t)(h[0] - l[0]) * (h[1] - l[1]) * (h[2] - l[2]);
}

// union of the slab boxes [s0, s1) (6 ints each); empty -> l > h
__device__ inline void slab_union(const int32_t *slab, int s0, int s1, int l[3], int h[3])
{
    for (int q = 0; q < 3; ++q) {
        l[q] = 0x7fffffff;
        h[q] = -0x7fffffff;
    }
    for (int s = s0; s < s1; ++s)
        for (int q = 0; q < 3; ++q) {
            l[q] = min(l[q], slab[6 * s + q]);
            h[q] = max(h[q], slab[6 * s + 3 + q]);
        }
}

__global__ __launch_bounds__(256) void k_kd_level_tight(KdArgs k)
{
    kd_priority();
    extern __shared__ int32_t slab[];   // [nbx + nby + nbz][6]
    __shared__ int32_t box[6];
    __shared__ int64_t cost[kMaxCand];
    __shared__ int64_t vnode;
    __shared__ int32_t choice[2];
    __shared__ int32_t child[2][6];
    __shared__ uint32_t scratch[5];
    __shared__ uint32_t last;
    const uint32_t begin = k.hdr->kd_begin, end = k.hdr->kd_end;
    if (begin == end) return;
    const int t = threadIdx.x;
    const int64_t vroot_prev = (int64_t)(((uint64_t)k.hdr->kd_vroot_hi << 32) | k.hdr->kd_vroot_lo);
    const int32_t *S = k.S;
    for (int64_t node = (int64_t)begin + blockIdx.x; node < end; node += gridDim.x) {
        if (t == 0) {
            if (node == 0) {
                for (int q = 0; q < 3; ++q) {
                    box[q] = k.lo[q];
                    box[3 + q] = k.hi[q];
                }
            } else {
                // child of the (r/2)-th splitting node of the level above
                const int64_t r = node - begin;
                const int64_t p = k.plist[r >> 1];
                const int32_t *cb = &k.clo[12 * p + 6 * (r & 1)];
                for (int q = 0; q < 6; ++q) box[q] = cb[q];
                for (int q = 0; q < 3; ++q) {
                    k.lo[3 * node + q] = box[q];
                    k.hi[3 * node + q] = box[3 + q];
                }
            }
        }
        __syncthreads();
        const int lo[3] = {box[0], box[1], box[2]}, hi[3] = {box[3], box[4], box[5]};
        const int e[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        const int off[3] = {0, e[0], e[0] + e[1]};
        const int nsl = e[0] + e[1] + e[2];
        for (int i = t; i < 6 * nsl; i += 256) slab[i] = (i % 6) < 3 ? 0x7fffffff : -0x7fffffff;
        __syncthreads();
        const int64_t bricks = (int64_t)e[0] * e[1] * e[2];
        for (int64_t i = t; i < bricks; i += 256) {
            const int c[3] = {lo[0] + (int)(i % e[0]), lo[1] + (int)((i / e[0]) % e[1]),
                              lo[2] + (int)(i / ((int64_t)e[0] * e[1]))};
            const int64_t b = c[0] + (int64_t)k.nb[0] * (c[1] + (int64_t)k.nb[1] * c[2]);
            if (!k.flags[b]) continue;
            const uint4 w = k.tbox[b];
            int l2[3], h2[3];
            unpack_box_u(w.x, w.y, w.z, l2, h2);
            if (!(h2[0] > l2[0] && h2[1] > l2[1] && h2[2] > l2[2])) continue;   // no visible cell
            for (int a = 0; a < 3; ++a) {
                int32_t *sl = &slab[6 * (off[a] + c[a] - lo[a])];
                for (int q = 0; q < 3; ++q) {
                    atomicMin(&sl[q], l2[q]);
                    atomicMax(&sl[3 + q], h2[q]);
                }
            }
        }
        __syncthreads();
        if (t == 0) {
            int l[3], h[3];
            slab_union(slab, 0, e[0], l, h);
            vnode = half_volume(l, h);
        }
        __syncthreads();
        const int64_t V = vnode;
        const int64_t vroot = node == 0 ? V : vroot_prev;
        const bool allowed = k.halting == 0 ? (10 * V > vroot) : (V > 512 * 8);
        int da = 0, dp = 0;
        const int ncand = allowed ? candidate(lo, hi, k.bins, -1, &da, &dp) : 0;
        if (t < ncand) {
            int a = 0, p = 0;
            candidate(lo, hi, k.bins, t, &a, &p);
            int l[3], h[3];
            slab_union(slab, off[a], off[a] + p - lo[a], l, h);
            int64_t c2 = half_volume(l, h);
            slab_union(slab, off[a] + p - lo[a], off[a] + e[a], l, h);
            cost[t] = c2 + half_volume(l, h);
        }
        __syncthreads();
        if (t == 0) {
            int axis = -1, plane = 0;
            if (ncand > 0) {
                int best = 0;
                for (int i = 1; i < ncand; ++i)
                    if (cost[i] < cost[best]) best = i;   // ties: the lower index
                if (cost[best] < V) {
                    candidate(lo, hi, k.bins, best, &axis, &plane);
                } else if (k.max_leaf > 0 && V > (int64_t)k.max_leaf * k.max_leaf * k.max_leaf * 8) {
                    // maximum leaf size: middle of the axis with the largest voxel extent
                    int64_t best_ext = -1;
                    for (int a = 0; a < 3; ++a) {
                        if (e[a] < 2) continue;
                        const int64_t ext = (int64_t)min(k.B * hi[a], k.n[a]) - (int64_t)k.B * lo[a];
                        if (ext > best_ext) {
                            best_ext = ext;
                            axis = a;
                            plane = lo[a] + e[a] / 2;
                        }
                    }
                }
            }
            choice[0] = axis;
            choice[1] = plane;
            if (node == 0) {
                k.hdr->kd_vroot_lo = (uint32_t)(uint64_t)V;
                k.hdr->kd_vroot_hi = (uint32_t)((uint64_t)V >> 32);
            }
        }
        __syncthreads();
        const int axis = choice[0], plane = choice[1];
        if (axis >= 0 && t < 12) {
            // the children: brick-tight boxes of the two sides (prefix count)
            const int side = t / 6, face = t % 6;
            int rl[3] = {lo[0], lo[1], lo[2]}, rh[3] = {hi[0], hi[1], hi[2]};
            if (side == 0) rh[axis] = plane; else rl[axis] = plane;
            child[side][face] = tight_face(k, S, rl, rh, face);
        }
        __syncthreads();
        if (t == 0) {
            k.axis[node] = axis;
            k.plane[node] = axis >= 0 ? plane : 0;
            k.split[node] = axis >= 0 ? 1 : 0;
            if (axis >= 0)
                for (int sd = 0; sd < 2; ++sd)
                    for (int f = 0; f < 6; ++f) k.clo[12 * node + 6 * sd + f] = child[sd][f];
            else
                k.first[node] = -1;
        }
        __syncthreads();   // box, slabs and shared results are reused by the next node
    }
    if (last_of_level(k, &last)) number_children(k, begin, end, scratch, nullptr);
}

// render box of node m from its brick box: voxels clipped to the volume, in
// half-voxel units
__device__ inline void kd_half_box(const KdArgs &k, int64_t m, int lo[3], int hi[3])
{
    for (int q = 0; q < 3; ++q) {
        lo[q] = 2 * (k.B * k.lo[3 * m + q]);
        hi[q] = 2 * min(k.B * k.hi[3 * m + q], k.n[q]);
    }
}

// voxel-tight leaves: the render box of a leaf is the union of the
// voxel-tight boxes of the non-empty bricks in it (one workgroup per leaf,
// grid-stride over the nodes).  Finished trees only, like k_kd_pack, which
// runs after it and takes the leaves' boxes from k.box.
__global__ __launch_bounds__(256) void k_kd_tight(KdArgs k)
{
    kd_priority();
    __shared__ int red[6];
    const uint32_t count = k.hdr->kd_count;
    if (k.hdr->kd_begin != k.hdr->kd_end || (int64_t)count > k.cap) return;
    for (int64_t m = blockIdx.x; m < (int64_t)count; m += gridDim.x) {
        if (k.axis[m] >= 0) continue;   // uniform per workgroup
        if (threadIdx.x < 6) red[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -1;
        __syncthreads();
        const int lo[3] = {k.lo[3 * m], k.lo[3 * m + 1], k.lo[3 * m + 2]};
        const int e[3] = {k.hi[3 * m] - lo[0], k.hi[3 * m + 1] - lo[1], k.hi[3 * m + 2] - lo[2]};
        const int64_t total = (int64_t)e[0] * e[1] * e[2];
        int tl[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, th[3] = {-1, -1, -1};
        for (int64_t t = threadIdx.x; t < total; t += 256) {
            const int bx = lo[0] + (int)(t % e[0]), by = lo[1] + (int)((t / e[0]) % e[1]),
                      bz = lo[2] + (int)(t / ((int64_t)e[0] * e[1]));
            const int64_t b = bx + (int64_t)k.nb[0] * (by + (int64_t)k.nb[1] * bz);
            if (!k.flags[b]) continue;
            const uint4 w = k.tbox[b];
            int l2[3], h2[3];
            unpack_box_u(w.x, w.y, w.z, l2, h2);
            for (int q = 0; q < 3; ++q) {
                tl[q] = min(tl[q], l2[q]);
                th[q] = max(th[q], h2[q]);
            }
        }
        for (int o = 32; o >= 1; o >>= 1)
            for (int q = 0; q < 3; ++q) {
                tl[q] = min(tl[q], __shfl_xor(tl[q], o, 64));
                th[q] = max(th[q], __shfl_xor(th[q], o, 64));
            }
        if ((threadIdx.x & 63) == 0)
            for (int q = 0; q < 3; ++q) {
                atomicMin(&red[q], tl[q]);
                atomicMax(&red[3 + q], th[q]);
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            // a leaf of a tight tree holds a non-empty brick; without one the
            // brick box stays (never the case for a finished tree)
            int l2[3], h2[3];
            kd_half_box(k, m, l2, h2);
            if (red[3] >= 0)
                for (int q = 0; q < 3; ++q) {
                    l2[q] = red[q];
                    h2[q] = red[3 + q];
                }
            uint32_t w[3];
            pack_box(l2, h2, w);
            k.box[m] = make_uint4(w[0], w[1], w[2], 0u);
        }
        __syncthreads();
    }
}

// traversal records: every node's render box, and an RNode per internal
// node.  Runs only on a finished tree: while levels remain (begin != end) the
// nodes of the pending level have not been evaluated, and their axis/first
// entries are stale workspace contents that must not be used as indices.
// With voxel-tight leaves, the leaves' boxes come from k_kd_tight.
__global__ __launch_bounds__(256) void k_kd_pack(KdArgs k)
{
    kd_priority();
    const uint32_t count = k.hdr->kd_count;
    if (k.hdr->kd_begin != k.hdr->kd_end || (int64_t)count > k.cap) return;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= (int64_t)count) return;
    int lo[3], hi[3];
    uint32_t w[3];
    const int a = k.axis[m];
    if (!(k.tight && a < 0)) {
        kd_half_box(k, m, lo, hi);
        pack_box(lo, hi, w);
        k.box[m] = make_uint4(w[0], w[1], w[2], 0u);
    }
    if (a < 0) return;
    const int c = k.first[m];
    if (c <= m || (int64_t)c + 1 >= (int64_t)count || a > 2) return;  // never true for a finished tree
    RNode rec;
    for (int side = 0; side < 2; ++side) {
        if (k.tight && k.axis[c + side] < 0) {
            const uint4 t = k.box[c + side];
            rec.w[3 * side] = t.x;
            rec.w[3 * side + 1] = t.y;
            rec.w[3 * side + 2] = t.z;
        } else {
            kd_half_box(k, c + side, lo, hi);
            pack_box(lo, hi, &rec.w[3 * side]);
        }
    }
    rec.w[6] = (uint32_t)c | ((uint32_t)a << 29) | (k.axis[c] < 0 ? kLeaf : 0u);
    rec.w[7] = (uint32_t)(c + 1) | (k.axis[c + 1] < 0 ? kLeaf : 0u);
    uint4 *dst = reinterpret_cast<uint4 *>(&k.rnode[m]);
    dst[0] = make_uint4(rec.w[0], rec.w[1], rec.w[2], rec.w[3]);
    dst[1] = make_uint4(rec.w[4], rec.w[5], rec.w[6], rec.w[7]);
}

}  // namespace

hipError_t launch_kd_pack(const KdArgs &k, int64_t max_nodes, hipStream_t s)
{
    if (max_nodes <= 0) return hipSuccess;
    if (k.tight)
        hipLaunchKernelGGL(k_kd_tight, dim3((unsigned)std::min<int64_t>(max_nodes, 2048)), dim3(256), 0, s, k);
    hipLaunchKernelGGL(k_kd_pack, dim3((unsigned)((max_nodes + 255) / 256)), dim3(256), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_kd_top(const KdArgs &k, hipStream_t s)
{
    hipLaunchKernelGGL(k_kd_top, dim3(1), dim3(64 * kKdTopWaves), 0, s, k);
    return hipGetLastError();
}

bool kd_projected(const KdArgs &k)
{
    return !k.tight_cost && k.nb[0] <= 32 && k.nb[1] <= 32 && k.nb[2] <= 32;
}

hipError_t launch_kd_root_bits(const KdArgs &k, hipStream_t s)
{
    hipLaunchKernelGGL(k_kd_root_bits, dim3(1), dim3(64), 0, s, k);
    return hipGetLastError();
}

bool kd_small(const KdArgs &k)
{
    return (int64_t)k.nb[0] * k.nb[1] * k.nb[2] <= kKdSmallBricks;
}

hipError_t launch_kd_prefix_root_small(const KdArgs &k, hipStream_t s)
{
    const size_t lds = sizeof(int32_t) * (size_t)k.nb[0] * k.nb[1] * k.nb[2];
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_kd_prefix_root_small),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kd_prefix_root_small, dim3(1), dim3(1024), lds, s, k);
    return hipGetLastError();
}

hipError_t launch_kd_levels(const KdArgs &k, int count, uint32_t first_launch, hipStream_t s)
{
    const int blocks = kd_level_blocks(k);
    if (k.tight_cost) {
        // per-slab unions of one node: 6 ints per brick slab of each axis
        const size_t lds = sizeof(int32_t) * 6 * ((size_t)k.nb[0] + k.nb[1] + k.nb[2]);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_kd_level_tight),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        for (int i = 0; i < count; ++i)
            hipLaunchKernelGGL(k_kd_level_tight, dim3(blocks), dim3(256), lds, s, k);
        return hipGetLastError();
    }
    for (int i = 0; i < count; ++i)
        hipLaunchKernelGGL(k_kd_level, dim3(blocks), dim3(256), 0, s, k, first_launch + (uint32_t)i);
    return hipGetLastError();
}

hipError_t launch_kd_prefix(const KdArgs &k, hipStream_t s)
{
    const int64_t lines[3] = {(int64_t)k.nb[1] * k.nb[2], (int64_t)k.nb[0] * k.nb[2],
                              (int64_t)k.nb[0] * k.nb[1]};
    for (int a = 0; a < 3; ++a)
        hipLaunchKernelGGL(k_prefix_axis, dim3((unsigned)((lines[a] + 255) / 256)), dim3(256), 0, s, k, a);
    return hipGetLastError();
}

hipError_t launch_kd_root(const KdArgs &k, hipStream_t s)
{
    hipLaunchKernelGGL(k_kd_root, dim3(1), dim3(64), 0, s, k);
    return hipGetLastError();
}


}  // namespace esk
