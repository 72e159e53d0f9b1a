// minmax.hip -- per-brick min/max of raw voxel values over each brick plus a
// one-voxel apron (the TF-independent half of brick classification; Sec. 2
// min-max range queries, Sec. 3.1 bricks).  HBM-bound: every voxel is read
// once per brick row it borders; the apron rows shared by neighbouring brick
// rows are re-read from L2 because neighbouring rows run on the same XCD.
//
// Work decomposition: one workgroup (4 waves) per (x segment, brick row by,
// brick slab bz).  A segment is 64 lanes x E voxels of one voxel row.  Each
// wave streams a quarter of the (B+2)^2 voxel rows of the window with 16-byte
// loads, keeping per-column min/max in registers (packed u16 / f16 min-max for
// the narrow types).  The four waves then meet in LDS, and one thread per
// brick reduces its B+2 columns (the apron columns at the segment edges come
// from two extra scalar loads per row).
#include "esk_internal.hpp"

namespace esk {
namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring brick rows (which share
// apron voxel rows) meet in the same L2.
__device__ inline int xcd_remap(int b, int G)
{
    if (G < 8) return b;
    int xcd = b & 7, per = G >> 3, rem = G & 7;
    return xcd * per + min(xcd, rem) + (b >> 3);
}

template <typename T> struct Acc;

template <> struct Acc<uint8_t> {
    static constexpr int E = 16, LOADS = 1;
    u16x2 mn[8], mx[8];
    __device__ void init()
    {
        for (int i = 0; i < 8; ++i) { mn[i] = u16x2{0xffff, 0xffff}; mx[i] = u16x2{0, 0}; }
    }
    __device__ void update(const uint4 *v)
    {
        const uint32_t w[4] = {v[0].x, v[0].y, v[0].z, v[0].w};
        for (int i = 0; i < 4; ++i) {
            u16x2 lo = __builtin_bit_cast(u16x2, w[i] & 0x00ff00ffu);
            u16x2 hi = __builtin_bit_cast(u16x2, (w[i] >> 8) & 0x00ff00ffu);
            mn[2 * i] = __builtin_elementwise_min(mn[2 * i], lo);
            mx[2 * i] = __builtin_elementwise_max(mx[2 * i], lo);
            mn[2 * i + 1] = __builtin_elementwise_min(mn[2 * i + 1], hi);
            mx[2 * i + 1] = __builtin_elementwise_max(mx[2 * i + 1], hi);
        }
    }
    // column e of this lane: word e/4, byte e%4 -> pair 2*(e/4) + (byte&1), element byte/2
    __device__ float cmin(int e) const { int b = e & 3; return (float)mn[2 * (e >> 2) + (b & 1)][b >> 1]; }
    __device__ float cmax(int e) const { int b = e & 3; return (float)mx[2 * (e >> 2) + (b & 1)][b >> 1]; }
};

template <> struct Acc<uint16_t> {
    static constexpr int E = 8, LOADS = 1;
    u16x2 mn[4], mx[4];
    __device__ void init()
    {
        for (int i = 0; i < 4; ++i) { mn[i] = u16x2{0xffff, 0xffff}; mx[i] = u16x2{0, 0}; }
    }
    __device__ void update(const uint4 *v)
    {
        const uint32_t w[4] = {v[0].x, v[0].y, v[0].z, v[0].w};
        for (int i = 0; i < 4; ++i) {
            u16x2 x = __builtin_bit_cast(u16x2, w[i]);
            mn[i] = __builtin_elementwise_min(mn[i], x);
            mx[i] = __builtin_elementwise_max(mx[i], x);
        }
    }
    __device__ float cmin(int e) const { return (float)mn[e >> 1][e & 1]; }
    __device__ float cmax(int e) const { return (float)mx[e >> 1][e & 1]; }
};

template <> struct Acc<_Float16> {
    static constexpr int E = 8, LOADS = 1;
    h16x2 mn[4], mx[4];
    __device__ void init()
    {
        const _Float16 pinf = __builtin_bit_cast(_Float16, (uint16_t)0x7c00);
        const _Float16 ninf = __builtin_bit_cast(_Float16, (uint16_t)0xfc00);
        for (int i = 0; i < 4; ++i) { mn[i] = h16x2{pinf, pinf}; mx[i] = h16x2{ninf, ninf}; }
    }
    __device__ void update(const uint4 *v)
    {
        const uint32_t w[4] = {v[0].x, v[0].y, v[0].z, v[0].w};
        for (int i = 0; i < 4; ++i) {
            h16x2 x = __builtin_bit_cast(h16x2, w[i]);
            mn[i] = __builtin_elementwise_min(mn[i], x);
            mx[i] = __builtin_elementwise_max(mx[i], x);
        }
    }
    __device__ float cmin(int e) const { return (float)mn[e >> 1][e & 1]; }
    __device__ float cmax(int e) const { return (float)mx[e >> 1][e & 1]; }
};

template <> struct Acc<float> {
    static constexpr int E = 8, LOADS = 2;
    float mn[8], mx[8];
    __device__ void init()
    {
        for (int i = 0; i < 8; ++i) { mn[i] = __builtin_inff(); mx[i] = -__builtin_inff(); }
    }
    __device__ void update(const uint4 *v)
    {
        const uint32_t w[8] = {v[0].x, v[0].y, v[0].z, v[0].w, v[1].x, v[1].y, v[1].z, v[1].w};
        for (int i = 0; i < 8; ++i) {
            float x = __builtin_bit_cast(float, w[i]);
            mn[i] = fminf(mn[i], x);
            mx[i] = fmaxf(mx[i], x);
        }
    }
    __device__ float cmin(int e) const { return mn[e]; }
    __device__ float cmax(int e) const { return mx[e]; }
};

template <typename T> __device__ inline float to_float(T v) { return (float)v; }

template <typename T> __device__ inline T from_float(float f) { return (T)f; }

// Loads the E voxels [xs, xs+E) of one row into uint4 words.  VEC: the row is
// 16-byte aligned and nx % E == 0, so the chunk is either whole or absent.
template <typename T, bool VEC>
__device__ inline void load_chunk(const T *row, int xs, int nx, uint4 *buf)
{
    constexpr int E = Acc<T>::E, LOADS = Acc<T>::LOADS;
    if (VEC) {
        if (xs < nx) {
            const uint4 *p = reinterpret_cast<const uint4 *>(row + xs);
            for (int l = 0; l < LOADS; ++l) buf[l] = p[l];
        } else {
            for (int l = 0; l < LOADS; ++l) buf[l] = make_uint4(0, 0, 0, 0);
        }
    } else {
        T tmp[E];
        for (int e = 0; e < E; ++e) tmp[e] = (xs + e < nx) ? row[xs + e] : (T)0;
        __builtin_memcpy(buf, tmp, sizeof(tmp));
    }
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_minmax(const T *__restrict__ vol, int nx, int ny, int nz,
                                                int B, int nbx, int nby, int nseg,
                                                T *__restrict__ outmin, T *__restrict__ outmax)
{
    constexpr int E = Acc<T>::E, LOADS = Acc<T>::LOADS, SEG = 64 * E, U = 4;
    __shared__ float smn[4][SEG], smx[4][SEG];
    __shared__ float emn[4][2], emx[4][2];

    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int seg = lb % nseg;
    const int rest = lb / nseg;
    const int by = rest % nby, bz = rest / nby;
    const int x0 = seg * SEG;
    const int y0 = max(0, by * B - 1), y1 = min(ny - 1, by * B + B);
    const int z0 = max(0, bz * B - 1), z1 = min(nz - 1, bz * B + B);
    const int ry = y1 - y0 + 1;
    const int R = ry * (z1 - z0 + 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int xs = x0 + lane * E;

    Acc<T> acc;
    acc.init();
    float eln = __builtin_inff(), elx = -__builtin_inff();
    float ern = __builtin_inff(), erx = -__builtin_inff();
    const bool has_left = (lane == 0) && x0 > 0;
    const bool has_right = (lane == 63) && (x0 + SEG) < nx;

    for (int r0 = wave; r0 < R; r0 += 4 * U) {
        uint4 buf[U][LOADS];
        float el[U], er[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 + 4 * u;
            el[u] = __builtin_inff();
            er[u] = __builtin_inff();
            if (r < R) {
                const int y = y0 + r % ry, z = z0 + r / ry;
                const T *row = vol + ((size_t)z * ny + y) * (size_t)nx;
                load_chunk<T, VEC>(row, xs, nx, buf[u]);
                if (has_left) el[u] = to_float(row[x0 - 1]);
                if (has_right) er[u] = to_float(row[x0 + SEG]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r0 + 4 * u < R) {
                acc.update(buf[u]);
                if (has_left) { eln = fminf(eln, el[u]); elx = fmaxf(elx, el[u]); }
                if (has_right) { ern = fminf(ern, er[u]); erx = fmaxf(erx, er[u]); }
            }
        }
    }

#pragma unroll
    for (int e = 0; e < E; ++e) {
        smn[wave][lane * E + e] = acc.cmin(e);
        smx[wave][lane * E + e] = acc.cmax(e);
    }
    if (lane == 0) { emn[wave][0] = eln; emx[wave][0] = elx; }
    if (lane == 63) { emn[wave][1] = ern; emx[wave][1] = erx; }
    __syncthreads();

    const int per_seg = SEG / B;
    const int j = threadIdx.x;
    if (j < per_seg) {
        const int bx = seg * per_seg + j;
        if (bx < nbx) {
            float mn = __builtin_inff(), mx = -__builtin_inff();
            const int c0 = j * B - 1, c1 = j * B + B;  // apron columns, segment-local
            for (int c = c0; c <= c1; ++c) {
                const int x = x0 + c;
                if (x < 0 || x >= nx) continue;
                for (int w = 0; w < 4; ++w) {
                    float a, b;
                    if (c < 0) { a = emn[w][0]; b = emx[w][0]; }
                    else if (c >= SEG) { a = emn[w][1]; b = emx[w][1]; }
                    else { a = smn[w][c]; b = smx[w][c]; }
                    mn = fminf(mn, a);
                    mx = fmaxf(mx, b);
                }
            }
            const size_t id = (size_t)bx + (size_t)nbx * ((size_t)by + (size_t)nby * bz);
            outmin[id] = from_float<T>(mn);
            outmax[id] = from_float<T>(mx);
        }
    }
}

template <typename T>
hipError_t launch_typed(const VolumeDesc &v, void *minv, void *maxv, hipStream_t s)
{
    constexpr int SEG = 64 * Acc<T>::E;
    const int nseg = (v.nx + SEG - 1) / SEG;
    const int64_t blocks = (int64_t)nseg * v.nb[1] * v.nb[2];
    if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const bool vec = (v.nx % Acc<T>::E == 0) && ((reinterpret_cast<uintptr_t>(v.vox) & 15) == 0);
    const T *vol = static_cast<const T *>(v.vox);
    if (vec)
        hipLaunchKernelGGL((k_minmax<T, true>), dim3((unsigned)blocks), dim3(256), 0, s, vol, v.nx, v.ny,
                           v.nz, v.B, v.nb[0], v.nb[1], nseg, (T *)minv, (T *)maxv);
    else
        hipLaunchKernelGGL((k_minmax<T, false>), dim3((unsigned)blocks), dim3(256), 0, s, vol, v.nx, v.ny,
                           v.nz, v.B, v.nb[0], v.nb[1], nseg, (T *)minv, (T *)maxv);
    return hipGetLastError();
}

// The blocked copy for the renderer, one workgroup per run of blocks along x
// of one (block row, block slab): the 81 voxel rows the run's stored blocks
// draw on (9 in y by 9 in z, edge rows repeated past the volume) are staged
// in LDS, then the run's blocks are written out as one contiguous stretch of
// 16-byte stores, so every cache line of the copy is written whole.  VEC:
// rows are read with 16-byte loads (nx a multiple of the 16-byte element
// count and a 16-byte aligned volume), else one element per load.
// Runs are 256 bytes of voxel row (measured against 128- and 512-byte runs:
// the 81 staged rows of a 512-byte run hold 43 KB of LDS and 3 workgroups
// per CU; 7-30 % slower).
template <typename T> constexpr int swz_run() { return 256 / (8 * (int)sizeof(T)); }

// Min/max summaries of a stored block (its 9^3 voxels, index l in 0..8 per
// axis), 8 minima then 8 maxima, summary m restricted to the layer l = 7 of
// every axis in m (bit 0: x, bit 1: y, bit 2: z).  The apron range of brick b
// along an axis, [bB - 1, bB + B] clamped to the volume, is exactly the full
// extent of the stored blocks bB/8 .. (b+1)B/8 - 1 plus the layer 7 of block
// bB/8 - 1 (B >= 8), so a brick's min/max combines these summaries (and the
// edge voxels repeated past the volume change neither).
template <typename T, bool VEC, bool SUM>
__global__ __launch_bounds__(256) void k_swizzle(const T *__restrict__ vol, int nx, int ny, int nz, int nqx,
                                                 int nqy, T *__restrict__ swz, float *__restrict__ blksum)
{
    constexpr int kSwzRun = swz_run<T>();
    constexpr int V = 16 / (int)sizeof(T);                       // elements per 16-byte access
    constexpr int X = kSwzRun * kSwzEdge + 1;                    // voxels of a staged row
    constexpr int W = (X + V - 1) / V * V;                       // staged row with padding
    constexpr int ROWS = kSwzSpan * kSwzSpan;
    __shared__ __align__(16) T tile[ROWS * W];
    const int qx0 = blockIdx.x * kSwzRun, qy = blockIdx.y, qz = blockIdx.z;
    const int nblk = min(kSwzRun, nqx - qx0);
    const int x0 = qx0 * kSwzEdge;
    // staged row r: voxel row y = min(8 qy + r % 9, ny - 1), z = min(8 qz + r / 9, nz - 1)
    auto row_ptr = [&](int r) {
        const int y = min(qy * kSwzEdge + r % kSwzSpan, ny - 1), z = min(qz * kSwzEdge + r / kSwzSpan, nz - 1);
        return vol + ((size_t)z * ny + y) * (size_t)nx;
    };
    if (VEC) {
        constexpr int CH = kSwzRun * kSwzEdge / V;   // 16-byte chunks per row
        for (int i = threadIdx.x; i < ROWS * CH; i += 256) {
            const int r = i / CH, c = i - r * CH;
            const int x = x0 + c * V;
            const T *row = row_ptr(r);
            if (x < nx) {
                *reinterpret_cast<uint4 *>(&tile[r * W + c * V]) = *reinterpret_cast<const uint4 *>(row + x);
            } else {
                const T e = row[nx - 1];   // past the volume: the edge voxel
                for (int k = 0; k < V; ++k) tile[r * W + c * V + k] = e;
            }
        }
        if (threadIdx.x < ROWS) {
            const int r = threadIdx.x;
            tile[r * W + X - 1] = row_ptr(r)[min(x0 + X - 1, nx - 1)];
        }
    } else {
        for (int i = threadIdx.x; i < ROWS * X; i += 256) {
            const int r = i / X, c = i - r * X;
            tile[r * W + c] = row_ptr(r)[min(x0 + c, nx - 1)];
        }
    }
    __syncthreads();
    if constexpr (SUM) {
        // each (block, row (lz, ly)): minimum/maximum over lx and the voxel
        // at lx = 7; then per block the summaries over all 81 rows, the 9
        // rows with ly = 7 or lz = 7, and the row with both
        constexpr int R81 = kSwzSpan * kSwzSpan;
        __shared__ float rmin[kSwzRun * R81], rmax[kSwzRun * R81], r7[kSwzRun * R81];
        for (int pr = threadIdx.x; pr < nblk * R81; pr += 256) {
            const int bb = pr / R81, r = pr - bb * R81;
            const T *row = &tile[r * W + bb * kSwzEdge];
            float rn = (float)row[0], rx = rn;
#pragma unroll
            for (int lx = 1; lx < kSwzSpan; ++lx) {
                const float q = (float)row[lx];
                rn = fminf(rn, q);
                rx = fmaxf(rx, q);
            }
            rmin[pr] = rn;
            rmax[pr] = rx;
            r7[pr] = (float)row[7];
        }
        __syncthreads();
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int b = wave; b < nblk; b += 4) {
            const int o = b * R81;
            // all rows: lanes take rows lane and lane + 64
            float a0 = rmin[o + lane], a1 = rmax[o + lane], a2 = r7[o + lane], a3 = a2;
            if (lane + 64 < R81) {
                a0 = fminf(a0, rmin[o + lane + 64]);
                a1 = fmaxf(a1, rmax[o + lane + 64]);
                a2 = fminf(a2, r7[o + lane + 64]);
                a3 = fmaxf(a3, r7[o + lane + 64]);
            }
            for (int d = 32; d >= 1; d >>= 1) {
                a0 = fminf(a0, __shfl_xor(a0, d, 64));
                a1 = fmaxf(a1, __shfl_xor(a1, d, 64));
                a2 = fminf(a2, __shfl_xor(a2, d, 64));
                a3 = fmaxf(a3, __shfl_xor(a3, d, 64));
            }
            // lanes 0..15 produce value i of the 16 (minima 0..7, maxima 8..15)
            const int m = lane & 7;
            const bool isMax = lane >= 8;
            float val;
            if (m == 0) val = isMax ? a1 : a0;
            else if (m == 1) val = isMax ? a3 : a2;
            else {
                // layers: m = 2, 3 (ly = 7) and 4, 5 (lz = 7) over 9 rows; 6, 7 one row
                const bool x7 = (m & 1) != 0;
                const float *src = x7 ? r7 : (isMax ? rmax : rmin);
                val = isMax ? -__builtin_inff() : __builtin_inff();
                const int cnt = m >= 6 ? 1 : kSwzSpan;
                for (int k = 0; k < cnt; ++k) {
                    const int r = m >= 6 ? 7 * kSwzSpan + 7 : (m < 4 ? k * kSwzSpan + 7 : 7 * kSwzSpan + k);
                    const float q = src[o + r];
                    val = isMax ? fmaxf(val, q) : fminf(val, q);
                }
            }
            if (lane < 16) blksum[((((size_t)qz * nqy + qy) * nqx + qx0 + b) << 4) + lane] = val;
        }
    }
    // the run's blocks are contiguous and kSwzBlock is a multiple of V, so the
    // stretch splits into whole 16-byte stores
    T *out = swz + (((size_t)qz * nqy + qy) * nqx + qx0) * kSwzBlock;
    const int total = nblk * kSwzBlock;
    for (int i = threadIdx.x * V; i < total; i += 256 * V) {
        // position of the chunk's first element, then stepped element by
        // element (x, then the 9x9 rows; past the 729th: padding)
        const int b = i / kSwzBlock, rem = i - b * kSwzBlock;
        int row = rem / kSwzSpan, lx = rem - row * kSwzSpan;   // row = lz * 9 + ly
        const int col0 = b * kSwzEdge;
        T v[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            v[e] = row < kSwzSpan * kSwzSpan ? tile[row * W + col0 + lx] : (T)0;
            const bool wrap = lx == kSwzSpan - 1;
            lx = wrap ? 0 : lx + 1;
            row = wrap ? row + 1 : row;
        }
        uint4 w;
        __builtin_memcpy(&w, v, 16);
        *reinterpret_cast<uint4 *>(out + i) = w;
    }
}

template <typename T>
hipError_t launch_swz_typed(const VolumeDesc &v, void *swz, float *blksum, hipStream_t s)
{
    static_assert(kSwzBlock % (16 / (int)sizeof(T)) == 0, "blocks split into 16-byte stores");
    constexpr int kSwzRun = swz_run<T>();
    const dim3 grid((unsigned)((v.nq[0] + kSwzRun - 1) / kSwzRun), (unsigned)v.nq[1], (unsigned)v.nq[2]);
    const bool vec = (v.nx % (16 / (int)sizeof(T)) == 0) && ((reinterpret_cast<uintptr_t>(v.vox) & 15) == 0);
    const T *vox = static_cast<const T *>(v.vox);
    T *out = static_cast<T *>(swz);
    if (vec && blksum)
        hipLaunchKernelGGL((k_swizzle<T, true, true>), grid, dim3(256), 0, s, vox, v.nx, v.ny, v.nz, v.nq[0], v.nq[1],
                           out, blksum);
    else if (vec)
        hipLaunchKernelGGL((k_swizzle<T, true, false>), grid, dim3(256), 0, s, vox, v.nx, v.ny, v.nz, v.nq[0],
                           v.nq[1], out, blksum);
    else if (blksum)
        hipLaunchKernelGGL((k_swizzle<T, false, true>), grid, dim3(256), 0, s, vox, v.nx, v.ny, v.nz, v.nq[0],
                           v.nq[1], out, blksum);
    else
        hipLaunchKernelGGL((k_swizzle<T, false, false>), grid, dim3(256), 0, s, vox, v.nx, v.ny, v.nz, v.nq[0],
                           v.nq[1], out, blksum);
    return hipGetLastError();
}

// Brick min/max from the stored blocks' summaries (B >= 8): every
// combination of "layer 7 of the block below" and "the core blocks" per axis
// (the lower layer only where the brick is not first); eight lanes per brick,
// one combination each, then a reduction over the eight.
template <typename T>
__global__ __launch_bounds__(256) void k_minmax_blocks(const float *__restrict__ blksum, int B, int nbx, int nby,
                                                       int nbz, int nq0, int nq1, int nq2, T *__restrict__ outmin,
                                                       T *__restrict__ outmax)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t id = t >> 3;
    const int m = (int)(t & 7);
    const bool live = id < (int64_t)nbx * nby * nbz;
    float mn = __builtin_inff(), mx = -__builtin_inff();
    if (live) {
        const int b[3] = {(int)(id % nbx), (int)((id / nbx) % nby), (int)(id / ((int64_t)nbx * nby))};
        const int nq[3] = {nq0, nq1, nq2};
        const int per = B / kSwzEdge;
        int c0[3], c1[3];
        for (int a = 0; a < 3; ++a) {
            c0[a] = b[a] * per;
            c1[a] = min(c0[a] + per, nq[a]);
        }
        if (!(((m & 1) && b[0] == 0) || ((m & 2) && b[1] == 0) || ((m & 4) && b[2] == 0))) {
            const int x0 = (m & 1) ? c0[0] - 1 : c0[0], x1 = (m & 1) ? c0[0] : c1[0];
            const int y0 = (m & 2) ? c0[1] - 1 : c0[1], y1 = (m & 2) ? c0[1] : c1[1];
            const int z0 = (m & 4) ? c0[2] - 1 : c0[2], z1 = (m & 4) ? c0[2] : c1[2];
            for (int qz = z0; qz < z1; ++qz)
                for (int qy = y0; qy < y1; ++qy)
                    for (int qx = x0; qx < x1; ++qx) {
                        const float *sm = blksum + ((((size_t)qz * nq1 + qy) * nq0 + qx) << 4);
                        mn = fminf(mn, sm[m]);
                        mx = fmaxf(mx, sm[8 + m]);
                    }
        }
    }
    // the brick's eight lanes are consecutive and aligned within the wave
    for (int o = 4; o >= 1; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o, 64));
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if (live && m == 0) {
        outmin[id] = from_float<T>(mn);
        outmax[id] = from_float<T>(mx);
    }
}

template <typename T>
hipError_t launch_mmb_typed(const VolumeDesc &v, const float *blksum, void *minv, void *maxv, hipStream_t s)
{
    const int64_t nb = (int64_t)v.nb[0] * v.nb[1] * v.nb[2];
    hipLaunchKernelGGL((k_minmax_blocks<T>), dim3((unsigned)((8 * nb + 255) / 256)), dim3(256), 0, s, blksum, v.B,
                       v.nb[0], v.nb[1], v.nb[2], v.nq[0], v.nq[1], v.nq[2], static_cast<T *>(minv),
                       static_cast<T *>(maxv));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_swizzle(const VolumeDesc &v, void *swz, float *blksum, hipStream_t s)
{
    switch (v.dtype) {
    case ESK_U8: return launch_swz_typed<uint8_t>(v, swz, blksum, s);
    case ESK_U16: return launch_swz_typed<uint16_t>(v, swz, blksum, s);
    case ESK_F16: return launch_swz_typed<_Float16>(v, swz, blksum, s);
    case ESK_F32: return launch_swz_typed<float>(v, swz, blksum, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_minmax_from_blocks(const VolumeDesc &v, const float *blksum, void *minv, void *maxv, hipStream_t s)
{
    if (v.B < kSwzEdge) return hipErrorInvalidValue;
    switch (v.dtype) {
    case ESK_U8: return launch_mmb_typed<uint8_t>(v, blksum, minv, maxv, s);
    case ESK_U16: return launch_mmb_typed<uint16_t>(v, blksum, minv, maxv, s);
    case ESK_F16: return launch_mmb_typed<_Float16>(v, blksum, minv, maxv, s);
    case ESK_F32: return launch_mmb_typed<float>(v, blksum, minv, maxv, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_minmax(const VolumeDesc &v, void *minv, void *maxv, hipStream_t s)
{
    switch (v.dtype) {
    case ESK_U8: return launch_typed<uint8_t>(v, minv, maxv, s);
    case ESK_U16: return launch_typed<uint16_t>(v, minv, maxv, s);
    case ESK_F16: return launch_typed<_Float16>(v, minv, maxv, s);
    case ESK_F32: return launch_typed<float>(v, minv, maxv, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace esk
