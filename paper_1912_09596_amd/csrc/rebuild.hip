// rebuild.hip -- per-TF rebuild up to the LBVH (Sec. 3.1): TF prefix count,
// brick classification + macrocell-grid bitmask, compaction, Morton codes,
// radix sort, Karras hierarchy, bottom-up AABB refit.
//
// All of this is O(bricks) and latency-bound at interactive sizes (tens of
// thousands of bricks), so kernels are few and wide: classification fuses the
// TF prefix count (each block rebuilds it in LDS from the TF copy), the grid
// bitmask (wave ballots) and the per-block non-empty counts; compaction fuses
// the Morton encoding; one workgroup sorts up to 32K keys entirely in LDS.
#include <algorithm>

#include "esk_internal.hpp"
#include "device_util.hpp"

namespace esk {
namespace {

__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}

// x -> bits 3i+2, y -> 3i+1, z -> 3i
__device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

__device__ inline uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// ---------------------------------------------------------------------------
// a2 + a3 + grid: classification
// ---------------------------------------------------------------------------

template <typename T> __device__ inline float raw(const void *p, int64_t i)
{
    return (float)static_cast<const T *>(p)[i];
}

// floor of x(v) = s(v) * (N-1); integer types exact, float types in FP32
// (this translation unit is compiled without FP contraction)
__device__ inline int tf_floor_index(float v, int dtype, float lo, float hi, int N)
{
    if (dtype == ESK_U8) return ((int)v * (N - 1)) / 255;
    if (dtype == ESK_U16) return ((int)v * (N - 1)) / 65535;
    float num = v - lo;
    float den = hi - lo;
    float s = num / den;
    s = s < 0.0f ? 0.0f : s;
    s = s > 1.0f ? 1.0f : s;
    float x = s * (float)(N - 1);
    return (int)floorf(x);
}

__device__ inline float load_minmax(const void *p, int dtype, int64_t i)
{
    switch (dtype) {
    case ESK_U8: return raw<uint8_t>(p, i);
    case ESK_U16: return raw<uint16_t>(p, i);
    case ESK_F16: return raw<_Float16>(p, i);
    default: return raw<float>(p, i);
    }
}

// ---------------------------------------------------------------------------
// per-voxel vote (Sec. 3.1's classification, an alternative to min/max): a
// brick is non-empty iff one of its own voxels maps to alpha > 0 under the
// renderer's TF lookup.  One workgroup per (256-voxel x run, brick row, brick
// slab); each lane tests its column of the brick's y-z cross-section, the
// lanes of one brick meet in a ballot, and one lane per brick raises the flag.
// Every voxel is read once: an HBM-bound pass per TF change.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_fill_u8(uint8_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

// Opacity of a TF entry as every kernel reads it: clamped to [0, 1], NaN as
// 0 (an opacity is a fraction; the caller's TF is not trusted to be one).
// Visibility (alpha > 0) is unchanged by the clamp.
__device__ inline float clean_alpha(float a) { return a > 0.0f ? fminf(a, 1.0f) : 0.0f; }

template <typename T>
__global__ __launch_bounds__(256) void k_vote(RebuildArgs a)
{
    __shared__ float alpha[kMaxTF];
    const int N = a.N;
    for (int i = threadIdx.x; i < N; i += 256) alpha[i] = clean_alpha(a.tf_src[4 * i + 3]);
    __syncthreads();
    const int B = a.vol.B, sh = a.vol.log2B;
    const int nx = a.vol.nx, ny = a.vol.ny, nz = a.vol.nz;
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int by = blockIdx.y, bz = blockIdx.z;
    const T *vol = static_cast<const T *>(a.vol.vox);
    bool vis = false;
    if (x < nx) {
        const int y1 = min(by * B + B, ny), z1 = min(bz * B + B, nz);
        for (int z = bz * B; z < z1 && !vis; ++z)
            for (int y = by * B; y < y1 && !vis; ++y) {
                const float v = (float)vol[((size_t)z * ny + y) * (size_t)nx + x];
                // the lookup of the renderer: s, x = s (N-1), lerp of alpha
                float t = (v - a.nlo) * a.nscale;
                t = fminf(fmaxf(t, 0.0f), 1.0f) * (float)(N - 1);
                const int i0 = min((int)t, N - 2);
                const float f = t - (float)i0;
                const float al = fmaf(f, alpha[i0 + 1] - alpha[i0], alpha[i0]);
                vis = al > 0.0f;
            }
    }
    // lanes x .. x+B-1 of one brick are consecutive within a wave (B divides 64)
    const uint64_t m = __ballot(vis);
    const int lane = threadIdx.x & 63;
    if ((lane & (B - 1)) == 0 && x < nx) {
        const uint64_t seg = (m >> lane) & (B == 64 ? ~0ull : ((1ull << B) - 1ull));
        if (seg) a.flags[(x >> sh) + (int64_t)a.vol.nb[0] * (by + (int64_t)a.vol.nb[1] * bz)] = 1;
    }
}

template <typename T> hipError_t launch_vote_typed(const RebuildArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)std::min<int64_t>((a.nb + 255) / 256, 4096)), dim3(256), 0, s,
                       a.flags, a.nb);
    const dim3 grid((unsigned)((a.vol.nx + 255) / 256), (unsigned)a.vol.nb[1], (unsigned)a.vol.nb[2]);
    hipLaunchKernelGGL((k_vote<T>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// voxel-tight brick boxes (the GPU k-d variant's per-macro-cell tight boxes,
// Sec. 3.2.2): a sample point p reads the trilinear cell c = floor(p - 1/2)
// (8 corner voxels, clamped), whose region is [c + 1/2, c + 3/2).  A cell is
// potentially visible iff the classification window of its own min/max holds
// an entry with alpha > 0; a brick's tight box is the bounding box of its
// potentially visible cells' regions, clipped to the brick, in half-voxel
// units.  Samples outside it read only invisible cells (alpha exactly 0).
// One workgroup per non-empty brick (grid-stride over the compacted ids); a
// brick without a visible cell gets a zero-volume box at its low corner.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_tight(RebuildArgs a)
{
    __shared__ int32_t P[kMaxTF + 1];
    __shared__ int red[6];
    const int N = a.N;
    for (int i = threadIdx.x; i <= N; i += 256) P[i] = a.tfP[i];
    const int n = (int)a.hdr->n;
    const int B = a.vol.B;
    const int nn[3] = {a.vol.nx, a.vol.ny, a.vol.nz};
    const uint32_t nbx = (uint32_t)a.vol.nb[0], nby = (uint32_t)a.vol.nb[1];
    const T *vol = static_cast<const T *>(a.vol.vox);
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t id = a.ids[i];
        const int bc[3] = {(int)(id % nbx), (int)((id / nbx) % nby), (int)(id / (nbx * nby))};
        int blo[3], bhi[3], ex[3];
        for (int q = 0; q < 3; ++q) {
            blo[q] = bc[q] * B;
            bhi[q] = min(blo[q] + B, nn[q]);
            ex[q] = bhi[q] - blo[q] + 1;   // cells blo-1 .. bhi-1
        }
        if (threadIdx.x < 6) red[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -1;
        __syncthreads();
        int tl[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, th[3] = {-1, -1, -1};
        const int cells = ex[0] * ex[1] * ex[2];
        for (int t = threadIdx.x; t < cells; t += 256) {
            const int c[3] = {blo[0] - 1 + t % ex[0], blo[1] - 1 + (t / ex[0]) % ex[1],
                              blo[2] - 1 + t / (ex[0] * ex[1])};
            int x0[3], x1[3];
            for (int q = 0; q < 3; ++q) {
                x0[q] = min(max(c[q], 0), nn[q] - 1);
                x1[q] = min(max(c[q] + 1, 0), nn[q] - 1);
            }
            float mn = 3.402823466e+38f, mx = -3.402823466e+38f;
            for (int corner = 0; corner < 8; ++corner) {
                const int x = (corner & 1) ? x1[0] : x0[0];
                const int y = (corner & 2) ? x1[1] : x0[1];
                const int z = (corner & 4) ? x1[2] : x0[2];
                const float v = (float)vol[((size_t)z * nn[1] + y) * (size_t)nn[0] + x];
                mn = fminf(mn, v);
                mx = fmaxf(mx, v);
            }
            const int lo = max(tf_floor_index(mn, a.vol.dtype, a.vlo, a.vhi, N) - 1, 0);
            const int hi = min(tf_floor_index(mx, a.vol.dtype, a.vlo, a.vhi, N) + 2, N - 1);
            if (P[hi + 1] - P[lo] <= 0) continue;
            for (int q = 0; q < 3; ++q) {
                tl[q] = min(tl[q], max(2 * c[q] + 1, 2 * blo[q]));
                th[q] = max(th[q], min(2 * c[q] + 3, 2 * bhi[q]));
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
            int l2[3], h2[3];
            const bool any = red[3] >= 0;
            for (int q = 0; q < 3; ++q) {
                l2[q] = any ? red[q] : 2 * blo[q];
                h2[q] = any ? red[3 + q] : 2 * blo[q];
            }
            uint32_t w[3];
            pack_box(l2, h2, w);
            a.tbox[id] = make_uint4(w[0], w[1], w[2], 0u);
        }
        __syncthreads();
    }
}

template <typename T> hipError_t launch_tight_typed(const RebuildArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_tight<T>), dim3((unsigned)std::min<int64_t>(a.nb, 4096)), dim3(256), 0, s, a);
    return hipGetLastError();
}

__device__ __forceinline__ void k_classify_body(const RebuildArgs &a, uint32_t bx)
{
    __shared__ int32_t P[kMaxTF + 1];
    __shared__ uint32_t scratch[8];
    __shared__ uint32_t wcount[16];
    const int N = a.N;
    // TF prefix count: 16 entries per thread
    {
        const int per = (N + 255) / 256;
        const int i0 = threadIdx.x * per;
        uint32_t c = 0;
        for (int i = i0; i < min(N, i0 + per); ++i) c += a.tf_src[4 * i + 3] > 0.0f ? 1u : 0u;
        uint32_t tot;
        uint32_t run = block_exclusive_scan<256>(c, scratch, &tot);
        for (int i = i0; i < min(N, i0 + per); ++i) {
            P[i] = (int32_t)run;
            run += a.tf_src[4 * i + 3] > 0.0f ? 1u : 0u;
        }
        if (threadIdx.x == 0) P[N] = (int32_t)tot;
        __syncthreads();
        if (bx == 0) {
            for (int i = threadIdx.x; i <= N; i += 256) a.tfP[i] = P[i];
            // the renderer's copy of the TF (both 16-byte aligned), opacity clamped
            for (int i = threadIdx.x; i < N; i += 256) {
                float4 e = reinterpret_cast<const float4 *>(a.tf_src)[i];
                e.w = clean_alpha(e.w);
                reinterpret_cast<float4 *>(a.tf)[i] = e;
            }
        }
    }
    const int64_t base = (int64_t)bx * kClassifyBlock;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < 4; ++j) {
        const int64_t b = base + 256 * j + threadIdx.x;
        int flag = 0;
        if (b < a.nb && a.vote) {
            flag = a.flags[b];
        } else if (b < a.nb) {
            float mn = load_minmax(a.minv, a.vol.dtype, b);
            float mx = load_minmax(a.maxv, a.vol.dtype, b);
            int lo = tf_floor_index(mn, a.vol.dtype, a.vlo, a.vhi, N) - 1;
            int hi = tf_floor_index(mx, a.vol.dtype, a.vlo, a.vhi, N) + 2;
            lo = max(lo, 0);
            hi = min(hi, N - 1);
            flag = (P[hi + 1] - P[lo]) > 0;
            a.flags[b] = (uint8_t)flag;
        }
        const uint64_t m = __ballot(flag);
        if (lane == 0) {
            const int64_t word = (base + 256 * j + 64 * wave) >> 5;
            a.grid[word] = (uint32_t)m;
            a.grid[word + 1] = (uint32_t)(m >> 32);
            wcount[4 * j + wave] = __popcll(m);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < 16; ++i) t += wcount[i];
        a.blkcnt[bx] = t;
    }
}

// exclusive scan of the per-block counts (single workgroup); total -> hdr->n
__device__ __forceinline__ void k_scan_blocks_body(uint32_t *cnt, int64_t nblk, DevHeader *hdr)
{
    __shared__ uint32_t scratch[17];
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t i0 = threadIdx.x * per;
    uint32_t c = 0;
    for (int64_t i = i0; i < min(nblk, i0 + per); ++i) c += cnt[i];
    uint32_t tot;
    uint32_t run = block_exclusive_scan<1024>(c, scratch, &tot);
    for (int64_t i = i0; i < min(nblk, i0 + per); ++i) {
        uint32_t t = cnt[i];
        cnt[i] = run;
        run += t;
    }
    if (threadIdx.x == 0) {
        hdr->n = tot;
        hdr->lbvh_height = 0;
    }
}

// a4 + a5: compaction in ascending brick id, with Morton keys
__global__ __launch_bounds__(256) void k_compact(RebuildArgs a)
{
    __shared__ uint32_t woff[16];
    const int64_t base = (int64_t)blockIdx.x * kClassifyBlock;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t *gw = a.grid + (base >> 5);
    if (threadIdx.x < 16) {
        // word pair of (j, wave) = 2*(4*j + wave) relative to the block
        const int q = threadIdx.x;
        woff[q] = __popc(gw[2 * q]) + __popc(gw[2 * q + 1]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = a.blkcnt[blockIdx.x];
        for (int q = 0; q < 16; ++q) {
            uint32_t t = woff[q];
            woff[q] = run;
            run += t;
        }
    }
    __syncthreads();
    for (int j = 0; j < 4; ++j) {
        const int q = 4 * j + wave;
        const uint64_t m = (uint64_t)gw[2 * q] | ((uint64_t)gw[2 * q + 1] << 32);
        if ((m >> lane) & 1ull) {
            const int64_t b = base + 64 * q + lane;
            const uint32_t pos = woff[q] + (uint32_t)__popcll(m & lanemask_lt());
            const uint32_t bx = (uint32_t)(b % a.vol.nb[0]);
            const uint32_t by = (uint32_t)((b / a.vol.nb[0]) % a.vol.nb[1]);
            const uint32_t bz = (uint32_t)(b / ((int64_t)a.vol.nb[0] * a.vol.nb[1]));
            a.ids[pos] = (uint32_t)b;
            a.keys[pos] = morton3(bx, by, bz);
        }
    }
}

// ---------------------------------------------------------------------------
// a4-a6 in Morton order: bricks lie on a grid, so enumerating the Morton
// codes of the brick grid in ascending order and keeping those of non-empty
// bricks yields the sorted keys directly -- the same array the radix sort
// produces (keys are unique), without sorting.  Used while the code domain
// 2^key_bits is at most 4x the brick count (near-cubic brick grids); one
// block per 1024 codes: count, scan of the block counts, scatter.
// ---------------------------------------------------------------------------
constexpr int kMortonBlock = 1024;

__device__ inline bool morton_flag(const RebuildArgs &a, uint32_t m)
{
    const uint32_t bx = compact3(m >> 2), by = compact3(m >> 1), bz = compact3(m);
    if (bx >= (uint32_t)a.vol.nb[0] || by >= (uint32_t)a.vol.nb[1] || bz >= (uint32_t)a.vol.nb[2]) return false;
    return a.flags[bx + (int64_t)a.vol.nb[0] * (by + (int64_t)a.vol.nb[1] * bz)] != 0;
}

__device__ __forceinline__ void k_morton_count_body(const RebuildArgs &a, uint32_t *cnt, int64_t codes, uint32_t bx)
{
    __shared__ uint32_t wcount[4];
    const int64_t base = (int64_t)bx * kMortonBlock;
    uint32_t c = 0;
    for (int j = 0; j < 4; ++j) {
        const int64_t m = base + 256 * j + threadIdx.x;
        const bool f = m < codes && morton_flag(a, (uint32_t)m);
        c += (uint32_t)__popcll(__ballot(f));
    }
    if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[bx] = wcount[0] + wcount[1] + wcount[2] + wcount[3];
}

// cnt: exclusive block offsets (k_scan_blocks)
__device__ __forceinline__ void k_morton_scatter_body(const RebuildArgs &a, const uint32_t *cnt, int64_t codes, uint32_t bx)
{
    __shared__ uint32_t woff[16];
    const int64_t base = (int64_t)bx * kMortonBlock;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool f[4];
    uint64_t mk[4];
    for (int j = 0; j < 4; ++j) {
        const int64_t m = base + 256 * j + threadIdx.x;
        f[j] = m < codes && morton_flag(a, (uint32_t)m);
        mk[j] = __ballot(f[j]);
        if (lane == 0) woff[4 * j + wave] = (uint32_t)__popcll(mk[j]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // codes ascend with j, then wave, then lane
        uint32_t run = cnt[bx];
        for (int q = 0; q < 16; ++q) {
            const uint32_t t = woff[q];
            woff[q] = run;
            run += t;
        }
    }
    __syncthreads();
    for (int j = 0; j < 4; ++j)
        if (f[j]) {
            const uint32_t pos = woff[4 * j + wave] + (uint32_t)__popcll(mk[j] & lanemask_lt());
            a.skeys[pos] = (uint32_t)(base + 256 * j + threadIdx.x);
        }
}

// ---------------------------------------------------------------------------
// a6: LSD radix sort of the Morton keys (ids are recovered from keys)
// ---------------------------------------------------------------------------

// LDS index with one pad word every 32 so that blocked per-thread access
// (thread t reads items t*I .. t*I+I-1) spreads over the banks
__device__ inline int padx(int i) { return i + (i >> 5); }

// Stable sort of n <= THREADS*ITEMS keys held in LDS `s` (padded indexing)
// by bits [bit0, bit0+nbits), two bits per pass (four buckets).
template <int THREADS, int ITEMS>
__device__ void lds_split_sort(uint32_t *s, int n, int bit0, int nbits, uint32_t *scratch)
{
    const int I = (n + THREADS - 1) / THREADS;  // items per thread this call
    const int first = threadIdx.x * I;
    const int cnt = max(0, min(I, n - first));
    for (int bit = bit0; bit < bit0 + nbits; bit += 2) {
        const int width = min(2, bit0 + nbits - bit);
        const uint32_t mask = (1u << width) - 1u;
        uint32_t k[ITEMS];
        uint32_t c01 = 0, c23 = 0;  // packed counts: buckets 0,1 in c01; 2,3 in c23 (16 bits each)
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            if (j < cnt) {
                k[j] = s[padx(first + j)];
                const uint32_t d = (k[j] >> bit) & mask;
                const uint32_t inc = 1u << (16 * (d & 1));
                if (d < 2) c01 += inc; else c23 += inc;
            }
        }
        uint32_t t01, t23;
        const uint32_t e01 = block_exclusive_scan<THREADS>(c01, scratch, &t01);
        const uint32_t e23 = block_exclusive_scan<THREADS>(c23, scratch, &t23);
        const uint32_t n0 = t01 & 0xffffu, n1 = t01 >> 16, n2 = t23 & 0xffffu;
        uint32_t off[4] = {e01 & 0xffffu, n0 + (e01 >> 16), n0 + n1 + (e23 & 0xffffu),
                           n0 + n1 + n2 + (e23 >> 16)};
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            if (j < cnt) {
                const uint32_t d = (k[j] >> bit) & mask;
                uint32_t p;
                // select without dynamic register indexing
                if (d == 0) p = off[0]++;
                else if (d == 1) p = off[1]++;
                else if (d == 2) p = off[2]++;
                else p = off[3]++;
                s[padx((int)p)] = k[j];
            }
        }
        __syncthreads();
    }
}

// single workgroup: sorts all n <= 32768 keys in LDS, writes sorted keys and ids
__global__ __launch_bounds__(1024) void k_sort_single(RebuildArgs a)
{
    extern __shared__ uint32_t s[];
    __shared__ uint32_t scratch[17];
    const int n = (int)a.hdr->n;
    for (int i = threadIdx.x; i < n; i += 1024) s[padx(i)] = a.keys[i];
    __syncthreads();
    lds_split_sort<1024, 32>(s, n, 0, a.key_bits, scratch);
    for (int i = threadIdx.x; i < n; i += 1024) a.skeys[i] = s[padx(i)];
}

// multi-block LSD pass, 8-bit digits: per-block histograms (digit-major)
__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t *in, const DevHeader *hdr, int bit,
                                                   uint32_t *hist, int64_t nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = hdr->n;
    const int64_t base = (int64_t)blockIdx.x * kSortBlockKeys;
    for (int i = threadIdx.x; i < kSortBlockKeys; i += 256) {
        const int64_t g = base + i;
        if (g < n) atomicAdd(&h[(in[g] >> bit) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan over the digit-major histogram (single workgroup), over the
// blocks that hold keys only: entry j of the scan is digit j / used of block
// j % used (blocks past the key count have empty histograms and no keys)
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *hist, const DevHeader *hdr, int64_t nblocks)
{
    __shared__ uint32_t scratch[17];
    const int64_t used = min(nblocks, ((int64_t)hdr->n + kSortBlockKeys - 1) / kSortBlockKeys);
    const int64_t len = 256 * used;
    const int64_t per = (len + 1023) / 1024;
    const int64_t i0 = threadIdx.x * per;
    const int64_t i1 = min(len, i0 + per);
    auto at = [&](int64_t j) -> uint32_t & { return hist[(j / used) * nblocks + j % used]; };
    uint32_t c = 0;
    for (int64_t j = i0; j < i1; ++j) c += at(j);
    uint32_t tot;
    uint32_t run = block_exclusive_scan<1024>(c, scratch, &tot);
    for (int64_t j = i0; j < i1; ++j) {
        uint32_t &h = at(j);
        const uint32_t t = h;
        h = run;
        run += t;
    }
}

// stable scatter: the block sorts its keys locally by the digit, then each key
// goes to (global offset of its digit in this block) + (rank inside the digit)
__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t *in, uint32_t *out,
                                                      const DevHeader *hdr, int bit,
                                                      const uint32_t *hist, int64_t nblocks)
{
    __shared__ uint32_t s[kSortBlockKeys + kSortBlockKeys / 32];
    __shared__ uint32_t scratch[5];
    __shared__ uint32_t start[256];
    const int64_t n = hdr->n;
    const int64_t base = (int64_t)blockIdx.x * kSortBlockKeys;
    const int cnt = (int)max((int64_t)0, min((int64_t)kSortBlockKeys, n - base));
    if (cnt == 0) return;
    for (int i = threadIdx.x; i < cnt; i += 256) s[padx(i)] = in[base + i];
    __syncthreads();
    lds_split_sort<256, 16>(s, cnt, bit, 8, scratch);
    // first local position of each digit
    start[threadIdx.x] = 0xffffffffu;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += 256) {
        const uint32_t d = (s[padx(i)] >> bit) & 255u;
        if (i == 0 || ((s[padx(i - 1)] >> bit) & 255u) != d) start[d] = (uint32_t)i;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += 256) {
        const uint32_t k = s[padx(i)];
        const uint32_t d = (k >> bit) & 255u;
        const uint32_t pos = hist[(int64_t)d * nblocks + blockIdx.x] + ((uint32_t)i - start[d]);
        out[pos] = k;
    }
}

// ---------------------------------------------------------------------------
// a7 + a8: Karras hierarchy, range-union AABBs, height
// ---------------------------------------------------------------------------

__device__ inline int delta(const uint32_t *k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    return __clz(k[i] ^ k[j]);
}

// one thread per key: leaf j gets its brick id and box; internal node i < n-1
// gets its children (Karras 2012: direction, range by doubling + binary
// search, split by binary search) and registers itself as their parent.
// Node numbering: internal i -> i, leaf j -> (n-1)+j.
// a8: AABBs.  Every internal node covers a contiguous range of sorted keys,
// so its children's boxes are unions over two leaf ranges: one wave per
// internal node reduces both ranges (no cross-node dependency, no atomics),
// writes the node's own box (the union) and its traversal record.  Ranges
// longer than a few chunks read the per-chunk unions (written by k_karras) for
// their whole chunks, so the few nodes near the root do not each stream
// every leaf.
constexpr int kLeafChunk = 256;

struct Box12 {
    int b[6];    // exported AABB (voxels): lo xyz, hi xyz
    int r[6];    // render box (half-voxel units): lo xyz, hi xyz
};

__device__ inline void box12_empty(Box12 &x)
{
    for (int q = 0; q < 3; ++q) {
        x.b[q] = x.r[q] = 0x7fffffff;
        x.b[3 + q] = x.r[3 + q] = -1;
    }
}

__device__ inline void box12_leaf(const RebuildArgs &a, int n, int j, Box12 &x)
{
    const int u = (n - 1) + j;
    int l2[3], h2[3];
    const uint4 w = a.lb_leafbox[j];
    unpack_box_u(w.x, w.y, w.z, l2, h2);
    for (int q = 0; q < 3; ++q) {
        x.b[q] = min(x.b[q], a.lb_lo[3 * u + q]);
        x.b[3 + q] = max(x.b[3 + q], a.lb_hi[3 * u + q]);
        x.r[q] = min(x.r[q], l2[q]);
        x.r[3 + q] = max(x.r[3 + q], h2[q]);
    }
}

__device__ inline void box12_wave(Box12 &x)
{
    for (int o = 32; o >= 1; o >>= 1)
        for (int q = 0; q < 3; ++q) {
            x.b[q] = min(x.b[q], __shfl_xor(x.b[q], o, 64));
            x.b[3 + q] = max(x.b[3 + q], __shfl_xor(x.b[3 + q], o, 64));
            x.r[q] = min(x.r[q], __shfl_xor(x.r[q], o, 64));
            x.r[3 + q] = max(x.r[3 + q], __shfl_xor(x.r[3 + q], o, 64));
        }
}

// Karras nodes and leaf boxes.  A block's 256 leaves are one chunk of
// kLeafChunk sorted keys: the block also writes the chunk's union boxes
// (read by k_lbvh_boxes for long ranges).
static_assert(kLeafChunk == 256, "one k_karras block per leaf chunk");
__device__ __forceinline__ void k_karras_body(const RebuildArgs &a, uint32_t bx)
{
    __shared__ int red[4][12];
    const int n = (int)a.hdr->n;
    const int i = bx * 256 + threadIdx.x;
    if ((int64_t)bx * kLeafChunk >= n) return;   // uniform per block
    const uint32_t *k = a.skeys;
    Box12 x;
    box12_empty(x);
    if (i < n) {
        const uint32_t key = k[i];
        const uint32_t bx = compact3(key >> 2), by = compact3(key >> 1), bz = compact3(key);
        a.sids[i] = bx + (uint32_t)a.vol.nb[0] * (by + (uint32_t)a.vol.nb[1] * bz);
        const int node = (n - 1) + i;
        const int b[3] = {(int)bx, (int)by, (int)bz};
        const int nn[3] = {a.vol.nx, a.vol.ny, a.vol.nz};
        int lo2[3], hi2[3];
        for (int q = 0; q < 3; ++q) {
            a.lb_lo[3 * node + q] = a.vol.B * b[q];
            a.lb_hi[3 * node + q] = min(a.vol.B * b[q] + a.vol.B, nn[q]);
            lo2[q] = 2 * a.lb_lo[3 * node + q];
            hi2[q] = 2 * a.lb_hi[3 * node + q];
        }
        // the leaf's render box: its brick, or the brick's voxel-tight box
        uint4 box;
        if (a.tight) {
            box = a.tbox[a.sids[i]];
        } else {
            uint32_t w[3];
            pack_box(lo2, hi2, w);
            box = make_uint4(w[0], w[1], w[2], 0u);
        }
        a.lb_leafbox[i] = box;
        if (n == 1) a.lb_root[0] = box;
        int l2[3], h2[3];
        unpack_box_u(box.x, box.y, box.z, l2, h2);
        for (int q = 0; q < 3; ++q) {
            x.b[q] = a.lb_lo[3 * node + q];
            x.b[3 + q] = a.lb_hi[3 * node + q];
            x.r[q] = l2[q];
            x.r[3 + q] = h2[q];
        }
    }
    // the chunk's union: waves, then the block
    box12_wave(x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int val = 0;   // lane q < 12 holds face q (selects: no dynamic register index)
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        val = lane == q ? x.b[q] : val;
        val = lane == 6 + q ? x.r[q] : val;
    }
    if (lane < 12) red[wave][lane] = val;
    __syncthreads();
    if (threadIdx.x < 12) {
        const int q = threadIdx.x, qq = q % 6;
        int v = red[0][q];
        for (int w = 1; w < 4; ++w) v = qq < 3 ? min(v, red[w][q]) : max(v, red[w][q]);
        a.lb_chunk[12 * (int64_t)bx + q] = v;
    }
    if (i >= n - 1) return;
    const int d = (delta(k, n, i, i + 1) - delta(k, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = delta(k, n, i, i - d);
    int lmax = 2;
    while (delta(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(k, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(k, n, i, j);
    int s = 0;
    for (int div = 2;; div <<= 1) {
        const int t = (l + div - 1) / div;
        if (delta(k, n, i, i + (s + t) * d) > dnode) s += t;
        if (t == 1) break;
    }
    const int g = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    const uint32_t left = (lo == g) ? (kLeaf | (uint32_t)g) : (uint32_t)g;
    const uint32_t right = (hi == g + 1) ? (kLeaf | (uint32_t)(g + 1)) : (uint32_t)(g + 1);
    a.lb_left[i] = left;
    a.lb_right[i] = right;
    const int hb = 31 - dnode;  // highest differing bit of the range
    a.lb_axis[i] = 2 - hb % 3;
    a.lb_parent[(left & kLeaf) ? (n - 1) + g : g] = (uint32_t)i;
    a.lb_parent[(right & kLeaf) ? (n - 1) + g + 1 : g + 1] = (uint32_t)i;
    a.lb_range[i] = make_int2(lo, hi);
}

__device__ __forceinline__ void k_lbvh_boxes_body(const RebuildArgs &a, uint32_t bx)
{
    const int n = (int)a.hdr->n;
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)bx * 4 + (threadIdx.x >> 6);
    if (i >= n - 1) return;
    const int2 rg = a.lb_range[i];
    const uint32_t l = a.lb_left[i], r = a.lb_right[i];
    const int g = (int)(l & ~kLeaf);
    int box[2][6], rbox[2][6];
    for (int side = 0; side < 2; ++side) {
        const int j0 = side == 0 ? rg.x : g + 1, j1 = side == 0 ? g : rg.y;
        Box12 x;
        box12_empty(x);
        if (j1 - j0 + 1 <= 4 * kLeafChunk) {
            for (int j = j0 + lane; j <= j1; j += 64) box12_leaf(a, n, j, x);
        } else {
            // leaves up to the first chunk boundary, whole chunks, leaves after the last
            const int c0 = (j0 + kLeafChunk - 1) / kLeafChunk, c1 = (j1 + 1) / kLeafChunk;
            for (int j = j0 + lane; j < c0 * kLeafChunk; j += 64) box12_leaf(a, n, j, x);
            for (int c = c0 + lane; c < c1; c += 64)
                for (int q = 0; q < 3; ++q) {
                    x.b[q] = min(x.b[q], a.lb_chunk[12 * c + q]);
                    x.b[3 + q] = max(x.b[3 + q], a.lb_chunk[12 * c + 3 + q]);
                    x.r[q] = min(x.r[q], a.lb_chunk[12 * c + 6 + q]);
                    x.r[3 + q] = max(x.r[3 + q], a.lb_chunk[12 * c + 9 + q]);
                }
            for (int j = c1 * kLeafChunk + lane; j <= j1; j += 64) box12_leaf(a, n, j, x);
        }
        box12_wave(x);
        for (int q = 0; q < 6; ++q) {
            box[side][q] = x.b[q];
            rbox[side][q] = x.r[q];
        }
    }
    if (lane == 0) {
        for (int q = 0; q < 3; ++q) {
            a.lb_lo[3 * i + q] = min(box[0][q], box[1][q]);
            a.lb_hi[3 * i + q] = max(box[0][3 + q], box[1][3 + q]);
        }
        if (i == 0) {
            int l2[3], h2[3];
            uint32_t w[3];
            for (int q = 0; q < 3; ++q) {
                l2[q] = min(rbox[0][q], rbox[1][q]);
                h2[q] = max(rbox[0][3 + q], rbox[1][3 + q]);
            }
            pack_box(l2, h2, w);
            a.lb_root[0] = make_uint4(w[0], w[1], w[2], 0u);
        }
        // A child subtree whose bricks fill its box (every brick of the box
        // non-empty) is traversed as one leaf with that box: its samples are
        // exactly those of its bricks, so the render and the counts do not
        // change.  Its box goes after the n leaf boxes, for popped links.
        // Not with voxel-tight leaf boxes (their union holds samples no leaf
        // box holds).
        uint32_t link[2] = {l, r};
        if (!a.tight) {
            const int B = a.vol.B;
            for (int side = 0; side < 2; ++side) {
                if (link[side] & kLeaf) continue;
                const int j0 = side == 0 ? rg.x : g + 1, j1 = side == 0 ? g : rg.y;
                int64_t bricks = 1;
                for (int q = 0; q < 3; ++q) bricks *= (int64_t)((box[side][3 + q] + B - 1) / B - box[side][q] / B);
                if (bricks == (int64_t)(j1 - j0 + 1)) {
                    uint32_t w[3];
                    pack_box(&rbox[side][0], &rbox[side][3], w);
                    a.lb_leafbox[n + (int64_t)link[side]] = make_uint4(w[0], w[1], w[2], 0u);
                    link[side] = kLeaf | (uint32_t)(n + (int64_t)link[side]);
                }
            }
        }
        RNode rec;
        pack_box(&rbox[0][0], &rbox[0][3], &rec.w[0]);
        pack_box(&rbox[1][0], &rbox[1][3], &rec.w[3]);
        rec.w[6] = link[0] | ((uint32_t)a.lb_axis[i] << 29);
        rec.w[7] = link[1];
        uint4 *dst = reinterpret_cast<uint4 *>(&a.lb_rnode[i]);
        dst[0] = make_uint4(rec.w[0], rec.w[1], rec.w[2], rec.w[3]);
        dst[1] = make_uint4(rec.w[4], rec.w[5], rec.w[6], rec.w[7]);
    }
}

// height in levels = 1 + the deepest leaf's number of ancestors
__device__ __forceinline__ void k_lbvh_height_body(const RebuildArgs &a, uint32_t bx)
{
    const int n = (int)a.hdr->n;
    const int j = bx * 256 + threadIdx.x;
    uint32_t depth = 0;
    if (j < n) {
        const int u = (n - 1) + j;
        if (n > 1) {
            uint32_t cur = a.lb_parent[u];
            depth = 1;
            while (cur != 0) {
                cur = a.lb_parent[cur];
                ++depth;
            }
        }
        depth += 1;
    }
    for (int o = 32; o >= 1; o >>= 1) depth = max(depth, (uint32_t)__shfl_xor((int)depth, o, 64));
    if ((threadIdx.x & 63) == 0 && depth > 0) atomicMax(&a.hdr->lbvh_height, depth);
}

// ---------------------------------------------------------------------------
// Kernel entry points.  Each body above runs either for one request (the
// arguments by value) or batched: blockIdx.y picks the request from a
// device array of arguments and the blocks past that request's own grid
// (the same count its single launch uses) exit at once.
// ---------------------------------------------------------------------------

__device__ inline int64_t morton_codes(const RebuildArgs &a) { return (int64_t)1 << a.key_bits; }
__device__ inline int64_t morton_blocks(const RebuildArgs &a) { return (morton_codes(a) + kMortonBlock - 1) / kMortonBlock; }

__global__ __launch_bounds__(256) void k_classify(RebuildArgs a) { k_classify_body(a, blockIdx.x); }
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *cnt, int64_t nblk, DevHeader *hdr)
{
    k_scan_blocks_body(cnt, nblk, hdr);
}
__global__ __launch_bounds__(256) void k_morton_count(RebuildArgs a, uint32_t *cnt, int64_t codes)
{
    k_morton_count_body(a, cnt, codes, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_morton_scatter(RebuildArgs a, const uint32_t *cnt, int64_t codes)
{
    k_morton_scatter_body(a, cnt, codes, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_karras(RebuildArgs a) { k_karras_body(a, blockIdx.x); }
__global__ __launch_bounds__(256) void k_lbvh_boxes(RebuildArgs a) { k_lbvh_boxes_body(a, blockIdx.x); }
__global__ __launch_bounds__(256) void k_lbvh_height(RebuildArgs a) { k_lbvh_height_body(a, blockIdx.x); }

// The batched launches run one flat grid: the requests' own grids laid end
// to end, off[r] = the first block of request r (off[n] = the total); a
// block finds its request by binary search over off (uniform, scalar loads).
__device__ inline int batch_request(const uint32_t *__restrict__ off, int n, uint32_t b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_classify_batch(const RebuildArgs *__restrict__ args,
                                                        const uint32_t *__restrict__ off, int n)
{
    const int r = batch_request(off, n, blockIdx.x);
    const RebuildArgs a = args[r];
    k_classify_body(a, blockIdx.x - off[r]);
}
// which = 0: the classification block counts (total -> hdr->n); 1: the
// Morton enumeration block counts.  One workgroup per request (blockIdx.y).
__global__ __launch_bounds__(1024) void k_scan_blocks_batch(const RebuildArgs *__restrict__ args, int which)
{
    const RebuildArgs a = args[blockIdx.y];
    if (which == 0) k_scan_blocks_body(a.blkcnt, a.nblk, a.hdr);
    else k_scan_blocks_body(a.hist, morton_blocks(a), a.hdr);
}
__global__ __launch_bounds__(256) void k_morton_count_batch(const RebuildArgs *__restrict__ args,
                                                            const uint32_t *__restrict__ off, int n)
{
    const int r = batch_request(off, n, blockIdx.x);
    const RebuildArgs a = args[r];
    k_morton_count_body(a, a.hist, morton_codes(a), blockIdx.x - off[r]);
}
__global__ __launch_bounds__(256) void k_morton_scatter_batch(const RebuildArgs *__restrict__ args,
                                                              const uint32_t *__restrict__ off, int n)
{
    const int r = batch_request(off, n, blockIdx.x);
    const RebuildArgs a = args[r];
    k_morton_scatter_body(a, a.hist, morton_codes(a), blockIdx.x - off[r]);
}
__global__ __launch_bounds__(256) void k_karras_batch(const RebuildArgs *__restrict__ args,
                                                      const uint32_t *__restrict__ off, int n)
{
    const int r = batch_request(off, n, blockIdx.x);
    const RebuildArgs a = args[r];
    k_karras_body(a, blockIdx.x - off[r]);
}
__global__ __launch_bounds__(256) void k_lbvh_boxes_batch(const RebuildArgs *__restrict__ args,
                                                          const uint32_t *__restrict__ off, int n)
{
    const int r = batch_request(off, n, blockIdx.x);
    const RebuildArgs a = args[r];
    k_lbvh_boxes_body(a, blockIdx.x - off[r]);
}
__global__ __launch_bounds__(256) void k_lbvh_height_batch(const RebuildArgs *__restrict__ args,
                                                           const uint32_t *__restrict__ off, int n)
{
    const int r = batch_request(off, n, blockIdx.x);
    const RebuildArgs a = args[r];
    k_lbvh_height_body(a, blockIdx.x - off[r]);
}

}  // namespace

hipError_t launch_vote(const RebuildArgs &a, hipStream_t s)
{
    switch (a.vol.dtype) {
    case ESK_U8: return launch_vote_typed<uint8_t>(a, s);
    case ESK_U16: return launch_vote_typed<uint16_t>(a, s);
    case ESK_F16: return launch_vote_typed<_Float16>(a, s);
    case ESK_F32: return launch_vote_typed<float>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tight(const RebuildArgs &a, hipStream_t s)
{
    switch (a.vol.dtype) {
    case ESK_U8: return launch_tight_typed<uint8_t>(a, s);
    case ESK_U16: return launch_tight_typed<uint16_t>(a, s);
    case ESK_F16: return launch_tight_typed<_Float16>(a, s);
    case ESK_F32: return launch_tight_typed<float>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_classify(const RebuildArgs &a, hipStream_t s)
{
    const unsigned blocks = (unsigned)a.nblk;
    hipLaunchKernelGGL(k_classify, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, a.blkcnt, a.nblk, a.hdr);
    return hipGetLastError();
}

hipError_t launch_compact(const RebuildArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact, dim3((unsigned)a.nblk), dim3(256), 0, s, a);
    return hipGetLastError();
}

bool sort_by_enumeration(const RebuildArgs &a)
{
    return ((int64_t)1 << a.key_bits) <= 4 * a.nb;
}

hipError_t launch_sort(const RebuildArgs &a, hipStream_t s)
{
    const int64_t codes = (int64_t)1 << a.key_bits;
    if (sort_by_enumeration(a)) {
        // sorted keys by enumeration; the block counts go to `hist` (the
        // sort's histogram, unused on this path: ceil(nb/4096)*256 entries
        // >= codes/1024 blocks)
        const unsigned blocks = (unsigned)((codes + kMortonBlock - 1) / kMortonBlock);
        hipLaunchKernelGGL(k_morton_count, dim3(blocks), dim3(256), 0, s, a, a.hist, codes);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, a.hist, (int64_t)blocks, a.hdr);
        hipLaunchKernelGGL(k_morton_scatter, dim3(blocks), dim3(256), 0, s, a, a.hist, codes);
        return hipGetLastError();
    }
    if (a.nb <= kSortSingleMax) {
        const size_t lds = sizeof(uint32_t) * (kSortSingleMax + kSortSingleMax / 32);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sort_single),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sort_single, dim3(1), dim3(1024), lds, s, a);
        return hipGetLastError();
    }
    // multi-block: ping-pong keys -> tmpkeys -> ... ending in skeys
    const int passes = (a.key_bits + 7) / 8;
    const uint32_t *src = a.keys;
    for (int p = 0; p < passes; ++p) {
        uint32_t *dst = ((passes - 1 - p) % 2 == 0) ? a.skeys : a.tmpkeys;
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)a.nsortblk), dim3(256), 0, s, src, a.hdr, 8 * p,
                           a.hist, a.nsortblk);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, a.hist, a.hdr, a.nsortblk);
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)a.nsortblk), dim3(256), 0, s, src, dst, a.hdr,
                           8 * p, a.hist, a.nsortblk);
        src = dst;
    }
    return hipGetLastError();
}

hipError_t launch_lbvh(const RebuildArgs &a, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.nb + 255) / 256);
    hipLaunchKernelGGL(k_karras, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_lbvh_boxes, dim3((unsigned)((a.nb + 3) / 4)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_lbvh_height, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rebuild_batch(const RebuildBatch &b, hipStream_t s)
{
    if (b.n_all > 0) {
        hipLaunchKernelGGL(k_classify_batch, dim3(b.blocks[0]), dim3(256), 0, s, b.all, b.off[0], b.n_all);
        hipLaunchKernelGGL(k_scan_blocks_batch, dim3(1, (unsigned)b.n_all), dim3(1024), 0, s, b.all, 0);
    }
    if (b.n_lbvh > 0) {
        hipLaunchKernelGGL(k_morton_count_batch, dim3(b.blocks[1]), dim3(256), 0, s, b.lbvh, b.off[1], b.n_lbvh);
        hipLaunchKernelGGL(k_scan_blocks_batch, dim3(1, (unsigned)b.n_lbvh), dim3(1024), 0, s, b.lbvh, 1);
        hipLaunchKernelGGL(k_morton_scatter_batch, dim3(b.blocks[1]), dim3(256), 0, s, b.lbvh, b.off[1], b.n_lbvh);
        hipLaunchKernelGGL(k_karras_batch, dim3(b.blocks[2]), dim3(256), 0, s, b.lbvh, b.off[2], b.n_lbvh);
        hipLaunchKernelGGL(k_lbvh_boxes_batch, dim3(b.blocks[3]), dim3(256), 0, s, b.lbvh, b.off[3], b.n_lbvh);
        hipLaunchKernelGGL(k_lbvh_height_batch, dim3(b.blocks[2]), dim3(256), 0, s, b.lbvh, b.off[2], b.n_lbvh);
    }
    return hipGetLastError();
}

int64_t rebuild_batch_blocks(const RebuildArgs &a, int kind)
{
    switch (kind) {
    case 0: return a.nblk;
    case 1: return (((int64_t)1 << a.key_bits) + kMortonBlock - 1) / kMortonBlock;
    case 2: return (a.nb + 255) / 256;
    case 3: return (a.nb + 3) / 4;
    }
    return 0;
}

}  // namespace esk
