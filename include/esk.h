/*
 * esk.h -- C ABI of the MI355X empty-space-skipping library.
 *
 * Implements the data-parallel hot path studied in "Comparing Hierarchical
 * Data Structures for Sparse Volume Rendering with Empty Space Skipping"
 * (Zellmann et al., arXiv 1912.09596): whenever the transfer function (TF)
 * changes, rebuild an empty-space-skipping hierarchy over a uniform scalar
 * volume (Sec. 1: the amount and arrangement of empty space change with the
 * alpha TF), then ray-march the volume, traversing the hierarchy to skip the
 * empty regions (Sec. 3, Sec. 4.1).
 *
 * Conventions
 *  - Voxel (x,y,z) of an nx*ny*nz volume lives at x + nx*(y + ny*z).
 *  - Bricks have edge B (a power of two, 4..32); brick (bx,by,bz) covers the
 *    voxels [B*b, min(B*b+B, n)) on each axis; its linear id is
 *    bx + nbx*(by + nby*bz) with nbx = ceil(nx/B) (likewise y, z).  At most 1024 bricks per
 *    axis (10 bits per axis of the 30-bit Morton code, Sec. 3.1), at most
 *    2^28 bricks in all, and at most 32767 voxels per axis (the renderer's
 *    boxes are uint16 in half-voxel units); beyond these limits calls return
 *    ESK_ELIMIT.
 *  - Transfer functions are N x RGBA float32, N in [2, 4096]; entry i sits at
 *    the normalised value i/(N-1).  Normalised value s(v): v/255 (u8),
 *    v/65535 (u16), clamp((v-lo)/(hi-lo), 0, 1) (f16, f32).  Every step
 *    reads an entry's opacity clamped to [0, 1], with NaN read as 0, so an
 *    entry is visible iff its alpha > 0; colour is used as given.
 *  - Images are H x W x RGBA float32, row 0 at the top, premultiplied colour.
 *  - Device pointers are HIP device addresses on the context's device.  All
 *    device memory is owned by the caller; the library borrows it and never
 *    allocates device memory (its one static device array, the argument
 *    staging of esk_render_batch_noalloc, is part of its code object).  Host
 *    pointers are plain host memory.
 *
 * Errors: every entry point returns an esk_status.  Arguments are validated on
 * the host before any device work is enqueued; a rejected call changes no
 * state.  Enqueued work is asynchronous on the context's stream; a device
 * fault surfaces as ESK_EDEVICE at the next call that synchronises
 * (esk_sync, esk_get_stats, esk_export, or a k-d rebuild).  esk_last_error
 * returns a human-readable reason for the last failure on a context.
 *
 * Threading: a context is used by one host thread at a time.
 */
#ifndef ESK_H
#define ESK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esk_ctx esk_ctx;

typedef enum {
    ESK_OK = 0,
    ESK_EINVAL = -1,    /* bad argument */
    ESK_ENOSPC = -2,    /* workspace smaller than esk_workspace_bytes() */
    ESK_ELIMIT = -3,    /* size beyond a documented limit (bricks/axis, TF entries) */
    ESK_EDEVICE = -4,   /* HIP runtime error or device fault */
    ESK_ESTATE = -5,    /* call out of order (no volume / no TF / accel not built) */
    ESK_EINTERNAL = -6
} esk_status;

typedef enum { ESK_U8 = 0, ESK_U16 = 1, ESK_F16 = 2, ESK_F32 = 3 } esk_dtype;

/* Acceleration structures.  Values are bits so a rebuild can build several. */
typedef enum {
    ESK_ACCEL_NONE = 0, /* full march, no skipping (the paper's "naive" column) */
    ESK_ACCEL_GRID = 1, /* uniform macrocell grid, macrocell = brick (Sec. 1) */
    ESK_ACCEL_LBVH = 2, /* LBVH over non-empty bricks (Sec. 3.1) */
    ESK_ACCEL_KD = 4,   /* binned k-d tree over brick occupancy (Sec. 3.2.2, 4.3) */
    ESK_ACCEL_HYBRID = 8 /* render only: traverse the k-d tree (built with ESK_ACCEL_KD,
                            typically shallow) and march each leaf with the macrocell
                            grid, skipping its empty bricks (the hybrid grid, Sec. 3.3) */
} esk_accel;

/* Classification mode, OR-ed into the build mask of
 * esk_set_transfer_function.  Default (bit clear): a brick is non-empty iff
 * the TF has an entry with alpha > 0 inside the index window of its value
 * range with apron (conservative: the skipped image equals the full march).
 * ESK_CLASSIFY_VOXEL: the per-voxel vote of Sec. 3.1 -- a brick is non-empty
 * iff one of its own voxels (no apron) maps to alpha > 0 under the
 * renderer's TF lookup in FP32 (s = (v - lo) * scale, x = clamp(s, 0, 1) *
 * (N-1), i0 = min(floor(x), N-2), alpha = fma(x - i0, a[i0+1] - a[i0],
 * a[i0])).  It reads every voxel per TF change and is not conservative:
 * interpolated samples between voxels can be visible in a brick whose voxels
 * are not, and such samples are skipped. */
enum { ESK_CLASSIFY_VOXEL = 0x100 };

/* Voxel-tight boxes, OR-ed into the build mask: after classification every
 * non-empty brick gets the bounding box of its potentially visible trilinear
 * cells (a cell -- the 8 voxels a sample reads -- is potentially visible iff
 * the classification window of its own min/max holds an entry with alpha > 0;
 * cell c covers [c + 1/2, c + 3/2) per axis), clipped to the brick, and the
 * LBVH leaves and the k-d leaves (union over their non-empty bricks) are
 * marched inside these boxes instead of whole bricks: the tight per-macro-
 * cell boxes of the GPU k-d builder of Sec. 3.2.2.  Samples outside read only
 * invisible cells, so every image still equals the full march.  Reads every
 * voxel of the non-empty bricks per TF change. */
enum { ESK_TIGHT_BOXES = 0x200 };

/* Voxel-tight split cost of the k-d build, OR-ed into the build mask with
 * ESK_ACCEL_KD (implies ESK_TIGHT_BOXES): the cost of a candidate plane is
 * the volume of the union of the voxel-tight boxes of the bricks left of it
 * plus that of the bricks right of it -- the GPU builder of Sec. 3.2.2,
 * which keeps one tight box per macro cell -- and every other volume the
 * build compares (the node's, against which a split must win; the root's,
 * for shallow halting; the 8^3-voxel and max_leaf^3 limits) is such a union
 * volume too.  Node regions, candidate planes, the maximum-leaf-size plane
 * and the children stay on the brick raster (brick-tight boxes). */
enum { ESK_KD_TIGHT_COST = 0x400 };

/* k-d build parameters (Sec. 4.3).
 *  halting:  0 = shallow: split only while 10*V(node) > V(root);
 *            1 = deep:    split only while V(node) > 8^3 voxels.
 *  max_leaf: 0 = off; else when the cost function says "leaf" and
 *            V(node) > max_leaf^3, split at the middle of the axis with the
 *            largest extent (the maximum-leaf-size rule).
 *  bins:     candidate planes lie on the bin boundaries lo + floor(j*e/bins),
 *            j = 1..bins-1, of the node's brick extent e on each axis
 *            (Sec. 3.2.2 uses 4); 2..16. */
typedef struct {
    int32_t halting;
    int32_t max_leaf;
    int32_t bins;
} esk_kd_params;

/* Camera basis, precomputed by the caller in FP32.  Pixel (x, y) has
 *   perspective:  origin eye,                    direction dir00 + (x+.5) du + (y+.5) dv
 *   orthographic: origin eye + (x+.5) du + (y+.5) dv, direction dir00
 * and the direction is normalised (Sec. 4.1 renders orthographic views; the
 * perspective form is the other common case). */
typedef struct {
    int32_t ortho;
    float eye[3];
    float dir00[3];
    float du[3];
    float dv[3];
} esk_camera;

typedef struct {
    int64_t n_bricks;    /* nbx*nby*nbz */
    int64_t n_nonempty;  /* bricks flagged by the last rebuild */
    int64_t lbvh_nodes;  /* 2N-1 (0 if N = 0), if the LBVH was built */
    int64_t kd_nodes;    /* k-d node count, if the k-d tree was built */
    int32_t lbvh_height; /* levels; a single leaf has height 1 */
    int32_t kd_height;
    int32_t nb[3];
    int32_t built;       /* esk_accel bits built by the last rebuild */
} esk_stats;

/* What esk_export copies out (all little-endian host arrays). */
typedef enum {
    ESK_X_MINMAX = 0,     /* 2*nb values in the volume dtype: all minima, then all maxima */
    ESK_X_TF_PREFIX = 1,  /* int32[N+1]: P[i] = #{j < i : alpha_j > 0} */
    ESK_X_FLAGS = 2,      /* uint8[nb]: 1 = brick may hold a visible sample */
    ESK_X_IDS = 3,        /* uint32[N]: non-empty brick ids, ascending */
    ESK_X_KEYS = 4,       /* uint32[N]: Morton keys of ESK_X_IDS, same order */
    ESK_X_SORTED_KEYS = 5,/* uint32[N]: keys ascending */
    ESK_X_SORTED_IDS = 6, /* uint32[N]: brick ids in sorted-key order (LBVH leaves) */
    ESK_X_LBVH_LEFT = 7,  /* uint32[N-1]: left child; bit 31 set = leaf index */
    ESK_X_LBVH_RIGHT = 8, /* uint32[N-1] */
    ESK_X_LBVH_AXIS = 9,  /* int32[N-1]: axis of the highest differing key bit */
    ESK_X_LBVH_LO = 10,   /* int32[N-1][3]: internal node AABB min, voxels */
    ESK_X_LBVH_HI = 11,   /* int32[N-1][3]: internal node AABB max (exclusive) */
    ESK_X_KD_LO = 12,     /* int32[M][3]: k-d node tight box min, bricks, BFS order */
    ESK_X_KD_HI = 13,     /* int32[M][3]: max (exclusive) */
    ESK_X_KD_AXIS = 14,   /* int32[M]: split axis, -1 = leaf */
    ESK_X_KD_PLANE = 15,  /* int32[M]: split plane in bricks (0 for leaves) */
    ESK_X_KD_FIRST = 16,  /* int32[M]: index of the left child (right = +1), -1 for leaves */
    ESK_X_GRID = 17,      /* uint32[ceil(nb/32)]: bit (i%32) of word i/32 = flag of brick i */
    ESK_X_TIGHT = 18      /* int32[nb][6]: voxel-tight box per brick in half-voxel units
                             (lo x,y,z, hi x,y,z; the box is [lo/2, hi/2)), zero for empty
                             bricks and bricks without a visible cell; needs ESK_TIGHT_BOXES */
} esk_export_what;

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  device = -1 creates a
 * validation-only context that checks arguments exactly as a device context
 * does and then returns ESK_ESTATE instead of touching any device.  The
 * context allocates pinned host memory for small read-backs only. */
esk_status esk_create(int device, void *hip_stream, esk_ctx **out);
esk_status esk_destroy(esk_ctx *ctx);

/* Pure host: bytes of device workspace esk_set_volume needs for this shape,
 * brick size and largest TF the caller will set. */
esk_status esk_workspace_bytes(int nx, int ny, int nz, int dtype, int brick, int max_tf_entries,
                               size_t *out);

/* Binds a volume and computes the per-brick min/max of raw values over each
 * brick plus a one-voxel apron (the trilinear footprint of the samples the
 * brick owns): the TF-independent half of classification (Sec. 2 min-max
 * range queries; Sec. 3.1 bricks).  d_vox: nx*ny*nz voxels of `dtype`;
 * value_lo < value_hi map f16/f32 values to [0,1] (ignored for u8/u16).
 * d_ws: caller-owned workspace of ws_bytes >= esk_workspace_bytes(...).
 * Both must stay alive (in stream order) until the next esk_set_volume or
 * esk_destroy.  Invalidates any previous TF/hierarchy. */
esk_status esk_set_volume(esk_ctx *ctx, const void *d_vox, int dtype, int nx, int ny, int nz,
                          float value_lo, float value_hi, int brick, int max_tf_entries,
                          void *d_ws, size_t ws_bytes);

/* Sets the TF and rebuilds (Sec. 3.1, 3.2.2): TF prefix count -> brick
 * classification (or the per-voxel vote with ESK_CLASSIFY_VOXEL) -> grid
 * bitmask -> compaction -> Morton codes in sorted order (by enumerating the
 * brick grid's codes, or a radix sort for lopsided grids) -> Karras hierarchy ->
 * AABB refit (if ESK_ACCEL_LBVH in build_mask), and the 3-D occupancy prefix
 * count -> level-synchronous binned k-d build (if ESK_ACCEL_KD).  The grid
 * is always built.  d_rgba: N x RGBA float32 on the device (16-byte
 * aligned), read by the enqueued work and copied into the workspace (the
 * caller may reuse it once the stream reaches this point).
 * kd may be NULL when ESK_ACCEL_KD is not requested.  Asynchronous: the
 * k-d build (and, when it is requested too, the LBVH build) runs on internal
 * streams of the context, forked from its stream after the classification;
 * a render of the LBVH waits for its build on the device, the k-d tree is
 * checked for completion (one synchronisation) when it is first used, and
 * the next esk_set_volume / esk_set_transfer_function waits for both. */
esk_status esk_set_transfer_function(esk_ctx *ctx, const float *d_rgba, int n_entries,
                                     int build_mask, const esk_kd_params *kd);

/* Batched rebuild: n requests (each a context with its own volume,
 * workspace and TF, all on one device) set their TFs and rebuild in one
 * launch chain on ctxs[0]'s stream: every kernel of the classification and
 * of the LBVH build (Sec. 3.1, a chain of O(n) kernels) runs once for all
 * requests, blockIdx.y picking the request.  Per-request semantics are
 * exactly those of esk_set_transfer_function(ctxs[i], d_tfs[i],
 * n_entries[i], build_mask, NULL), so every hierarchy is bit-identical to
 * rebuilding it alone.  build_mask: ESK_ACCEL_GRID and/or ESK_ACCEL_LBVH (no
 * k-d tree, vote or tight boxes: ESK_EINVAL).  The batch takes the sorted
 * keys of every request from the Morton enumeration while its code domain
 * is at most 2^20 codes (or 4x its brick count); larger lopsided grids are
 * classified in the batch and finish their LBVH (compaction, radix sort,
 * nodes) with launches of their own inside this call.  Each context appears once.  Every context's
 * earlier work must be ordered before this call (same stream, or
 * synchronised by the caller); a pending k-d build of any of them is waited
 * for on ctxs[0]'s stream.  d_args: caller-owned device buffer of
 * esk_rebuild_batch_bytes(n) bytes, 16-byte aligned, reusable once the
 * stream has passed this call.  n in [1, 65535]. */
esk_status esk_rebuild_batch_bytes(int n, size_t *out);
esk_status esk_rebuild_batch(esk_ctx *const *ctxs, int n, const float *const *d_tfs, const int *n_entries,
                             int build_mask, void *d_args, size_t args_bytes);

/* Renders W x H pixels with `accel` (ESK_ACCEL_NONE, or one structure built by
 * the last rebuild): emission-absorption ray marching with post-classification
 * and no early ray termination or shading (Sec. 4.1).  Samples lie at
 * t_k = t0 + (k+1/2)*step along each ray, t0 = max(0, volume entry); a sample
 * at p counts iff p is in [0,n)^3; its value is the cell-centred trilinear
 * interpolation (clamp to edge), looked up in the TF with linear
 * interpolation; alpha is corrected to 1-(1-a)^(step/opacity_ref_step)
 * (opacity_ref_step = 0: no correction) and composited front to back.
 * Skipping never changes the image: skipped samples have alpha exactly 0.
 * d_rgba_out: H*W*4 float32.  d_count_out (nullable): H*W int32, the number of
 * samples composited per pixel. */
esk_status esk_render(esk_ctx *ctx, int accel, const esk_camera *cam, int width, int height,
                      float step, float opacity_ref_step, float *d_rgba_out, int32_t *d_count_out);

/* Several frames of one context in one call (Sec. 4.1, as esk_render per
 * frame), typically one view rendered with several structures: frame i is
 * exactly esk_render(ctx, accels[i], &cams[i], widths[i], heights[i], step,
 * opacity_ref_step, d_outs[i], d_counts ? d_counts[i] : NULL).  The frames
 * of the k-d tree (and hybrid), of the LBVH and of the other modes run on
 * three streams (the context's internal build streams and its own), so the
 * kernels of different structures overlap; every frame is complete on the
 * context's stream when the work enqueued after this call runs, as after n
 * esk_render calls.  The frames that need no k-d tree are enqueued first;
 * a k-d or hybrid frame follows once the host has seen the k-d build finish
 * (its height sizes the traversal stack, as in esk_render), while the others
 * already run.  Frames must not share an output.  n in [1,
 * ESK_RENDER_MULTI_MAX].  All frames are checked before any is enqueued; a
 * frame failing after the checks (a device error, a k-d tree too tall)
 * leaves the frames before it enqueued and joined. */
#define ESK_RENDER_MULTI_MAX 8

/* The stream (a hipStream_t) on which esk_render_multi runs the frames of
 * `accel` outside a graph capture: for timing or ordering against them only
 * (events recorded there around a call bracket that call's frames of
 * `accel`).  Work the caller enqueues there runs in order with the
 * context's builds and frames. */
esk_status esk_render_stream(esk_ctx *ctx, int accel, void **stream_out);
esk_status esk_render_multi(esk_ctx *ctx, int n, const int *accels, const esk_camera *cams, const int *widths,
                            const int *heights, float step, float opacity_ref_step, float *const *d_outs,
                            int32_t *const *d_counts);

/* Batched rendering: n requests (each a context with its own volume, TF and
 * hierarchy, all of the same volume dtype and on one device) rendered by one
 * kernel launch on ctxs[0]'s stream, request i into d_outs[i] (heights[i] x
 * widths[i] x RGBA float32), with accel, step and opacity_ref_step shared.
 * Per-request semantics are exactly those of esk_render, so each image is
 * bit-identical to rendering it alone.  Every context's earlier work must be
 * ordered before this call (same stream, or synchronised by the caller).
 * d_args: caller-owned device buffer of esk_render_batch_bytes(n) bytes,
 * 16-byte aligned, that receives the per-request arguments; it may be reused
 * once the stream has passed this call.  n in [1, 65535]. */
esk_status esk_render_batch_bytes(int n, size_t *out);
esk_status esk_render_batch(esk_ctx *const *ctxs, int n, int accel, const esk_camera *cams, const int *widths,
                            const int *heights, float step, float opacity_ref_step, float *const *d_outs,
                            void *d_args, size_t args_bytes);

/* Allocation-free batched rendering, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): esk_render_batch without the caller's argument buffer.  The
 * per-request arguments go to a static device array inside the library, one
 * per device, of at most 1024 requests (n above that returns ESK_ELIMIT and
 * enqueues nothing); the call allocates nothing (no device, host or pinned
 * memory): the array's device address, a pinned host staging of the same
 * size and an upload event are set up once per device by the first
 * esk_create on it and held until the process ends.  Validation, semantics
 * and results are exactly those of esk_render_batch (bit-identical images).
 * Every call on a device shares that device's array and staging, which keep
 * the last call's arguments: successive calls must be ordered on one stream
 * (or the caller waits for the previous batch to finish); calls that overlap
 * on one device -- from several host threads, or on different streams while
 * an earlier batch may still read its arguments -- race. */
esk_status esk_render_batch_noalloc(esk_ctx *const *ctxs, int n, int accel, const esk_camera *cams,
                                    const int *widths, const int *heights, float step, float opacity_ref_step,
                                    float *const *d_outs);

/* Waits for the context's stream and its internal build streams, and
 * finishes a k-d build whose speculative batch of level launches fell short
 * of the tree (more levels are enqueued and waited for), so every structure
 * built by the last esk_set_transfer_function is complete on return; reports
 * device faults. */
esk_status esk_sync(esk_ctx *ctx);

/* Synchronises and fills *out. */
esk_status esk_get_stats(esk_ctx *ctx, esk_stats *out);

/* Synchronises and copies one array of the current state into `host`
 * (capacity cap bytes); *used receives the byte count (also when cap is too
 * small, which returns ESK_ENOSPC).  ESK_X_IDS and ESK_X_KEYS: where the
 * last rebuild did not need them (no voxel-tight boxes, sorted keys by
 * enumeration) the export first enqueues the compaction (Sec. 3.1) of the
 * current flags on the context's stream. */
esk_status esk_export(esk_ctx *ctx, int what, void *host, size_t cap, size_t *used);

const char *esk_strerror(esk_status s);
const char *esk_last_error(const esk_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ESK_H */
