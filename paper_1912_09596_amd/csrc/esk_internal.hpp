// esk_internal.hpp -- shared between the host runtime (api.cpp) and the HIP
// kernel translation units of libesk.  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/esk.h"

namespace esk {

constexpr int kMaxTF = 4096;          // TF entries the ABI accepts
constexpr int kMaxBricksPerAxis = 1024;  // 10 bits per axis of the 30-bit Morton code
constexpr int kMaxVoxelsPerAxis = 32767; // render boxes are uint16 in half-voxel units
constexpr uint32_t kLeaf = 0x80000000u;
constexpr int kClassifyBlock = 1024;  // bricks per classification / compaction block
constexpr int kSortSingleMax = 32768; // keys one workgroup sorts in LDS
constexpr int kSortBlockKeys = 4096;  // keys per block of the multi-block sort
// Batched rebuilds take the sorted keys from the Morton enumeration while the
// code domain is at most this many codes (or 4x the brick count, the rule of
// a single rebuild): one launch chain for every request instead of a sort
// per request.  The enumeration's 1024-code block counts go to `hist`, which
// the workspace sizes for it.
constexpr int64_t kBatchEnumCodes = (int64_t)1 << 20;
constexpr int kMaxKdStack = 128;      // deepest k-d tree the renderer traverses
constexpr int64_t kMaxBricks = (int64_t)1 << 28;  // node indices fit the 29-bit fields of RNode
constexpr uint32_t kIndexMask = 0x1fffffffu;

// Traversal record of one internal node (32 bytes, two 16-byte loads): the
// boxes of both children in half-voxel units (uint16, half-open: the box is
// [lo/2, hi/2), so voxel-tight boxes with bounds on cell boundaries fit; at
// most 32767 voxels per axis) and the children, each with bit 31 = leaf;
// bits 29..30 of c0 hold this node's split axis.  Packed leaf and root boxes
// (uint4: the same three words and a zero) use the same units.
struct RNode {
    uint32_t w[8];  // lo0.x|lo0.y, lo0.z|hi0.x, hi0.y|hi0.z, lo1.x|lo1.y, lo1.z|hi1.x, hi1.y|hi1.z, c0, c1
};

// Small device-resident state written by the rebuild kernels.
struct DevHeader {
    uint32_t n;            // non-empty bricks
    uint32_t lbvh_height;  // levels
    uint32_t kd_count;     // k-d nodes emitted so far
    uint32_t kd_height;    // levels emitted so far
    uint32_t kd_begin;     // current level [begin, end)
    uint32_t kd_end;
    uint32_t kd_ticket;    // blocks of the current k-d level launch that finished
    uint32_t kd_vroot_lo;  // voxel-tight split cost: the root's union volume
    uint32_t kd_vroot_hi;  //   (half-voxel units, 64 bits)
    // what k-d level launch i finds in slot i % 2 (the launch before it wrote it):
    // {kKdNumbered, begin, end}: evaluate the level [begin, end), its parents listed in plist;
    // {kKdToNumber, begin, end}: the level [begin, end) was evaluated, its children are not numbered yet
    uint32_t kd_next[2][3];
    uint32_t kd_top_levels;  // levels the first (single-workgroup) k-d launch evaluated
    uint32_t pad[48];
};
static_assert(sizeof(DevHeader) == 256, "header is one 256-byte slot");
constexpr uint32_t kKdNumbered = 1, kKdToNumber = 2;

// Byte offsets of every array inside the caller's workspace.
struct Layout {
    int64_t nb;            // bricks
    int64_t nblk;          // classification blocks
    int64_t nsortblk;      // multi-block sort blocks
    size_t header, swz, blksum, minv, maxv, tf, tfP, flags, grid, blkcnt;
    size_t ids, keys, skeys, tmpkeys, sids, hist;
    size_t tbox;           // voxel-tight box per brick (half-voxel units, packed)
    size_t lb_left, lb_right, lb_axis, lb_parent, lb_lo, lb_hi, lb_range, lb_rnode, lb_leafbox, lb_root, lb_chunk;
    size_t kd_S, kd_lo, kd_hi, kd_axis, kd_plane, kd_first, kd_split, kd_clo, kd_plist, kd_rnode, kd_box;
    size_t total;
};

Layout make_layout(int nx, int ny, int nz, int brick, int elem_bytes, int max_tf);

int elem_size(int dtype);

// ---- launchers (each enqueues on `s`; returns hipSuccess or the launch error)
// The renderer samples a copy of the volume stored in 8^3-voxel blocks, made
// at esk_set_volume: the 2x2x2 footprints of the 64 rays of a wave then fall
// into a few blocks instead of dozens of voxel rows.  A stored block holds
// the 9^3 voxels from its corner (its own 8^3 and the first voxel of the next
// block along each axis, edge voxels repeated past the volume), x fastest,
// then y, then z, padded to 736 elements (a multiple of 16 bytes for every
// element type); blocks x-fastest.  All 8 neighbours of a sample then lie in
// one stored block at fixed offsets.
constexpr int kSwzEdge = 8;     // voxels per block edge
constexpr int kSwzSpan = 9;     // stored voxels per block edge
constexpr int kSwzBlock = 736;  // stored elements per block (9^3 = 729, padded)
inline int64_t swz_bytes(const int nq[3], int elem_bytes)
{
    return (int64_t)nq[0] * nq[1] * nq[2] * kSwzBlock * elem_bytes;
}

struct VolumeDesc {
    const void *vox;
    int dtype, nx, ny, nz, B, log2B, nb[3];
    const void *swz;       // blocked copy in the workspace
    int nq[3];             // blocks per axis (ceil(n / 8))
};

hipError_t launch_minmax(const VolumeDesc &v, void *minv, void *maxv, hipStream_t s);
// blksum: null, or 16 floats per stored block receiving its min/max summaries
// (for launch_minmax_from_blocks; bricks of 8 voxels or more)
hipError_t launch_swizzle(const VolumeDesc &v, void *swz, float *blksum, hipStream_t s);
hipError_t launch_minmax_from_blocks(const VolumeDesc &v, const float *blksum, void *minv, void *maxv,
                                     hipStream_t s);

struct RebuildArgs {
    VolumeDesc vol;
    float vlo, vhi;
    int N;                 // TF entries
    float *tf;             // workspace copy (written by k_classify, read by the renderer)
    const float *tf_src;   // the caller's TF (read by the vote and k_classify)
    int32_t *tfP;
    const void *minv, *maxv;
    uint8_t *flags;
    uint32_t *grid;
    uint32_t *blkcnt;
    uint32_t *ids, *keys, *skeys, *tmpkeys, *sids, *hist;
    uint32_t *lb_left, *lb_right, *lb_parent;
    int32_t *lb_axis, *lb_lo, *lb_hi;
    int2 *lb_range;        // [first, last] sorted-key range of each internal node
    RNode *lb_rnode;
    uint4 *lb_leafbox;
    DevHeader *hdr;
    int64_t nb, nblk, nsortblk;
    int key_bits;          // Morton bits that can be non-zero
    int vote;              // 1: flags come from the per-voxel vote (k_vote), not min/max
    float nlo, nscale;     // the renderer's value normalisation s = (v - nlo) * nscale
    int tight;             // 1: render boxes of LBVH leaves are the voxel-tight boxes
    uint4 *tbox;           // per brick: packed voxel-tight box (written by k_tight)
    uint4 *lb_root;        // packed render box of the LBVH root
    int32_t *lb_chunk;     // per chunk of 256 sorted leaves: union boxes (6 voxel + 6 half-voxel ints)
};

hipError_t launch_vote(const RebuildArgs &a, hipStream_t s);
hipError_t launch_tight(const RebuildArgs &a, hipStream_t s);
// classification, grid bitmask and block counts (hdr->n)
hipError_t launch_classify(const RebuildArgs &a, hipStream_t s);
// ids of the non-empty bricks in ascending id, with their Morton keys (after launch_classify)
hipError_t launch_compact(const RebuildArgs &a, hipStream_t s);
// the sorted keys come from enumerating the brick grid's Morton codes (no sort, no compaction input)
bool sort_by_enumeration(const RebuildArgs &a);
hipError_t launch_sort(const RebuildArgs &a, hipStream_t s);
hipError_t launch_lbvh(const RebuildArgs &a, hipStream_t s);
// Many requests in one launch chain: classification (+ block scan) of the
// n_all requests of `all`, then the Morton enumeration and the LBVH kernels
// of the n_lbvh requests of `lbvh` (device arrays of arguments).  Each
// batched kernel runs the requests' own grids end to end in one flat grid:
// off[k] (device, n + 1 entries) holds the first block of every request for
// block-count kind k (0 classification, 1 Morton enumeration, 2 Karras /
// height, 3 boxes; rebuild_batch_blocks gives the count), blocks[k] the total.
struct RebuildBatch {
    const RebuildArgs *all, *lbvh;
    int n_all, n_lbvh;
    const uint32_t *off[4];
    unsigned blocks[4];
};
hipError_t launch_rebuild_batch(const RebuildBatch &b, hipStream_t s);
int64_t rebuild_batch_blocks(const RebuildArgs &a, int kind);

struct KdArgs {
    int nb[3], B, n[3];
    const uint8_t *flags;
    const uint32_t *grid;  // the same flags as a bitmask (bit b of word b / 32, b the linear brick id)
    int32_t *S;
    int32_t *lo, *hi, *axis, *plane, *first, *split, *clo;  // clo: [node][side][6 faces]
    int32_t *plist;        // the splitting nodes of the last level, in order (parents of the next level)
    RNode *rnode;
    uint4 *box;
    DevHeader *hdr;
    int halting, max_leaf, bins;
    int64_t cap;           // node capacity of the k-d arrays (2 nb)
    int tight;             // 1: leaf render boxes are unions of the bricks' voxel-tight boxes
    const uint4 *tbox;     // per brick: packed voxel-tight box
    int tight_cost;        // 1: split cost and compared volumes from the unions of the voxel-tight boxes
};

bool kd_projected(const KdArgs &k);
hipError_t launch_kd_root_bits(const KdArgs &k, hipStream_t s);
hipError_t launch_kd_top(const KdArgs &k, hipStream_t s);
bool kd_small(const KdArgs &k);
hipError_t launch_kd_prefix_root_small(const KdArgs &k, hipStream_t s);
hipError_t launch_kd_prefix(const KdArgs &k, hipStream_t s);
hipError_t launch_kd_root(const KdArgs &k, hipStream_t s);
hipError_t launch_kd_levels(const KdArgs &k, int count, uint32_t first_launch, hipStream_t s);
hipError_t launch_kd_pack(const KdArgs &k, int64_t max_nodes, hipStream_t s);

struct RenderArgs {
    VolumeDesc vol;
    float vlo, vscale;     // s = clamp((v - vlo) * vscale, 0, 1)
    const float *tf;
    int N;
    esk_camera cam;
    int W, H;
    float dt, expo;
    int correct;
    float *out;
    int32_t *count;
    const uint32_t *grid;
    const uint4 *lb_root;
    const RNode *lb_rnode;
    const uint4 *lb_leafbox;
    const RNode *kd_rnode;
    const uint4 *kd_box;
    const DevHeader *hdr;
    int stack_cap;
    int ctx, cty;          // the tile the volume's centre projects to (dispatch starts there)
    int seg_len;           // lattice samples per ray segment of a split tile
};

// Render workgroups cover one 8x8-pixel tile (fine-grained scheduling
// balances the very uneven per-tile work, and small images still spread over
// every CU; 16x16 tiles measured the same for the trees at 1080p and up to
// 3x slower at 128x128).  A workgroup holds kRaySegments waves: the sample
// sequence of every ray of a long tile is split into that many consecutive
// segments, one per wave, composited separately and combined front to back,
// so a tile whose rays cross much non-empty space no longer bounds the whole
// frame on one wave's instruction stream; a short tile keeps one wave and the
// other ends at once.  Every mode splits alike.
constexpr int kRaySegments = 2;
// a tile is split in S = clamp(K / seg_len, 1, kRaySegments) segments, K the
// lattice samples of its longest ray; seg_len is kRaySegLen for images of
// at least kRaySegFewTiles tiles, else kRaySegLenFew: few tiles leave most
// SIMDs idle, so shorter rays split too (measured: 128^2 to 256^2 renders
// 25-40 % faster; for 512^2 requests batched 64 to a launch the extra waves
// cost 5-8 %, hence the threshold).  It depends on the image size only, so a
// request renders the same alone and in a batch.  kRaySegLen: 192 measured
// 1 % faster than 256 for the three 1080p frames of one view rendered
// together (128: between; 512 and 1024: 2 and 5 % slower).
constexpr int kRaySegLen = 192;
constexpr int kRaySegLenFew = 32;
constexpr int kRaySegFewTiles = 2048;
__host__ __device__ constexpr int render_tile_for(int) { return 8; }
__host__ __device__ constexpr int render_threads_for(int) { return 64 * kRaySegments; }

// dynamic LDS of one render workgroup: [TF (N <= 1024)][traversal stack]
__host__ __device__ constexpr size_t render_lds_bytes(int accel, int N, bool tf_lds, int stack_cap)
{
    return (tf_lds ? (size_t)N * 16 : 0) + (size_t)stack_cap * render_threads_for(accel) * sizeof(int);
}

hipError_t launch_render(int accel, const RenderArgs &r, hipStream_t s);

// Allocation-free batched rendering: the per-request arguments live in a
// static device array of kNoAllocBatchMax entries (one per device, shared by
// every call on it); noalloc_init resolves its address (with `device`
// current) and allocates the pinned host staging and the upload event once
// per device; noalloc_slot returns the slot, or null before a successful init.
constexpr int kNoAllocBatchMax = 1024;
struct NoAllocSlot {
    RenderArgs *d_args = nullptr;     // device address of the static array
    RenderArgs *h_staging = nullptr;  // pinned host staging of the same size
    hipEvent_t done = nullptr;        // recorded after the last upload from h_staging
    bool recorded = false;
};
hipError_t noalloc_init(int device);
NoAllocSlot *noalloc_slot(int device);

// n requests of one accel and volume dtype; d_args: n RenderArgs in device memory
hipError_t launch_render_batch(int accel, int dtype, const RenderArgs *d_args, int n, int tiles_x, int tiles_y,
                               size_t lds, bool narrow, bool tfl, hipStream_t s);

}  // namespace esk
