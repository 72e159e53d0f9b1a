// api.cpp -- host runtime behind include/esk.h: argument validation,
// workspace layout, and the stream-ordered orchestration of the kernels.
// All argument checks run on the host before any device call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "esk_internal.hpp"

#include <rocprofiler-sdk-roctx/roctx.h>

namespace esk {

int elem_size(int dtype)
{
    switch (dtype) {
    case ESK_U8: return 1;
    case ESK_U16: return 2;
    case ESK_F16: return 2;
    case ESK_F32: return 4;
    }
    return 0;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Layout make_layout(int nx, int ny, int nz, int brick, int elem_bytes, int max_tf)
{
    Layout L;
    std::memset(&L, 0, sizeof(L));
    const int nbx = (nx + brick - 1) / brick, nby = (ny + brick - 1) / brick, nbz = (nz + brick - 1) / brick;
    const int64_t nb = (int64_t)nbx * nby * nbz;
    const int nq[3] = {(nx + kSwzEdge - 1) / kSwzEdge, (ny + kSwzEdge - 1) / kSwzEdge, (nz + kSwzEdge - 1) / kSwzEdge};
    L.nb = nb;
    L.nblk = (nb + kClassifyBlock - 1) / kClassifyBlock;
    L.nsortblk = (nb + kSortBlockKeys - 1) / kSortBlockKeys;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    const size_t n4 = (size_t)nb * 4;
    L.header = take(sizeof(DevHeader));
    L.swz = take((size_t)swz_bytes(nq, elem_bytes));
    // min/max summaries per stored block: FP32 volumes with bricks of 8 or more
    L.blksum = take(elem_bytes == 4 && brick >= kSwzEdge ? (size_t)nq[0] * nq[1] * nq[2] * 16 * sizeof(float) : 0);
    L.minv = take((size_t)nb * elem_bytes);
    L.maxv = take((size_t)nb * elem_bytes);
    L.tf = take((size_t)max_tf * 16);
    L.tfP = take((size_t)(max_tf + 1) * 4);
    L.flags = take((size_t)nb);
    L.grid = take((size_t)L.nblk * (kClassifyBlock / 32) * 4);
    L.blkcnt = take((size_t)L.nblk * 4);
    L.ids = take(n4);
    L.keys = take(n4);
    L.skeys = take(n4);
    L.tmpkeys = take(n4);
    L.sids = take(n4);
    // radix-sort histograms, or the block counts of a Morton enumeration of
    // up to max(4 nb, kBatchEnumCodes) codes (1024 codes per block)
    L.hist = take((size_t)std::max<int64_t>(L.nsortblk * 256, kBatchEnumCodes / 1024) * 4);
    L.lb_left = take(n4);
    L.lb_right = take(n4);
    L.lb_axis = take(n4);
    L.lb_parent = take(2 * n4);
    L.lb_lo = take(2 * n4 * 3);
    L.lb_hi = take(2 * n4 * 3);
    L.lb_range = take(2 * n4);
    L.lb_rnode = take((size_t)nb * sizeof(RNode));
    L.lb_leafbox = take((size_t)nb * 2 * 16);   // leaf boxes, then boxes of subtrees traversed as one leaf
    L.lb_root = take(16);
    L.lb_chunk = take((size_t)((nb + 255) / 256) * 48);
    L.tbox = take((size_t)nb * 16);
    L.kd_S = take(n4);
    L.kd_lo = take(2 * n4 * 3);
    L.kd_hi = take(2 * n4 * 3);
    L.kd_axis = take(2 * n4);
    L.kd_plane = take(2 * n4);
    L.kd_first = take(2 * n4);
    L.kd_split = take(2 * n4);
    L.kd_clo = take(2 * n4 * 12);
    L.kd_plist = take(2 * n4);
    L.kd_rnode = take(2 * (size_t)nb * sizeof(RNode));
    L.kd_box = take(2 * (size_t)nb * 16);
    L.total = off;
    return L;
}

}  // namespace esk

using namespace esk;

struct esk_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    DevHeader *pinned = nullptr;   // host read-back slot
    std::string err;
    // volume
    bool has_volume = false;
    VolumeDesc vol{};
    float vlo = 0.f, vhi = 1.f;
    int max_tf = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout L{};
    // TF / hierarchy
    bool has_tf = false;
    int N = 0;
    int built = 0;
    bool tight = false;         // render boxes are voxel-tight (ESK_TIGHT_BOXES)
    uint32_t kd_height = 0;
    uint32_t kd_count = 0;
    bool kd_on_device = false;  // k-d build enqueued; completion and height not yet read back
    esk_kd_params kd_params{1, 0, 4};
    bool kd_tight_cost = false; // the last k-d build used the voxel-tight split cost
    // host staging of batched render arguments (pinned; reused once the
    // previous upload has completed)
    RenderArgs *staging = nullptr;
    int staging_cap = 0;
    hipEvent_t staging_done = nullptr;
    // the same for batched rebuild arguments
    RebuildArgs *rb_staging = nullptr;
    int rb_staging_cap = 0;
    hipEvent_t rb_done = nullptr;
    int kd_level_hint = 24;     // levels enqueued per rebuild (adapts to the last height)
    int kd_levels_enqueued = 0;
    // the k-d build runs on an auxiliary stream forked after classification,
    // so its latency-bound level launches overlap work on the main stream
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_kd = nullptr;
    DevHeader *pinned_kd = nullptr;   // header snapshot taken at the end of the k-d build
    bool kd_joined = true;            // main stream already ordered after the last k-d build
    // the LBVH build runs on a second auxiliary stream forked at the same
    // point, so the grid render starts right after classification
    hipStream_t aux2 = nullptr;
    hipEvent_t ev_lbvh = nullptr;
    hipEvent_t ev_join[2] = {nullptr, nullptr};  // esk_render_multi: the frames on aux2 / aux done
    bool lbvh_joined = true;          // main stream already ordered after the last LBVH build
    bool rebuild_compacts = false;    // the last rebuild (and any replay of it) writes ids/keys
};

namespace {

esk_status fail(esk_ctx *c, esk_status s, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

esk_status hip_check(esk_ctx *c, hipError_t e, const char *what)
{
    if (e == hipSuccess) return ESK_OK;
    return fail(c, ESK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool valid_brick(int b) { return b == 4 || b == 8 || b == 16 || b == 32; }

int log2i(int b)
{
    int l = 0;
    while ((1 << l) < b) ++l;
    return l;
}

int bits_for(int n)  // bits to index [0, n)
{
    int b = 0;
    while ((1 << b) < n) ++b;
    return b;
}

esk_status check_shape(esk_ctx *c, int nx, int ny, int nz, int dtype, int brick, int max_tf)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(c, ESK_EINVAL, "dims must be >= 1 (got %d %d %d)", nx, ny, nz);
    if (nx > kMaxVoxelsPerAxis || ny > kMaxVoxelsPerAxis || nz > kMaxVoxelsPerAxis)
        return fail(c, ESK_ELIMIT, "more than %d voxels on an axis (%d %d %d)", kMaxVoxelsPerAxis, nx, ny, nz);
    if (elem_size(dtype) == 0) return fail(c, ESK_EINVAL, "unknown dtype %d", dtype);
    if (!valid_brick(brick)) return fail(c, ESK_EINVAL, "brick must be 4, 8, 16 or 32 (got %d)", brick);
    if (max_tf < 2 || max_tf > kMaxTF)
        return fail(c, ESK_ELIMIT, "max_tf_entries must be in [2, %d] (got %d)", kMaxTF, max_tf);
    const int nbx = (nx + brick - 1) / brick, nby = (ny + brick - 1) / brick, nbz = (nz + brick - 1) / brick;
    if (nbx > kMaxBricksPerAxis || nby > kMaxBricksPerAxis || nbz > kMaxBricksPerAxis)
        return fail(c, ESK_ELIMIT, "more than %d bricks on an axis (%d %d %d)", kMaxBricksPerAxis, nbx, nby, nbz);
    if ((int64_t)nbx * nby * nbz > kMaxBricks)
        return fail(c, ESK_ELIMIT, "more than %lld bricks", (long long)kMaxBricks);
    return ESK_OK;
}

bool finite3(const float *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

template <typename T> T *at(esk_ctx *c, size_t off) { return reinterpret_cast<T *>(c->ws + off); }

esk_status read_header(esk_ctx *c)
{
    hipError_t e = hipMemcpyAsync(c->pinned, at<DevHeader>(c, c->L.header), sizeof(DevHeader),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_check(c, e, "reading device header");
}

// true while `s` is being captured into a graph: the host staging of the
// batched calls is then neither waited for nor marked (nothing executes
// during a capture; a replay re-reads the staging the capture recorded)
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

// orders the main stream after the last k-d build (before anything that
// reads its results or rewrites the arrays it reads)
esk_status join_kd(esk_ctx *c)
{
    if (c->kd_joined) return ESK_OK;
    hipError_t e = hipStreamWaitEvent(c->stream, c->ev_kd, 0);
    if (e != hipSuccess) return hip_check(c, e, "joining the k-d stream");
    c->kd_joined = true;
    return ESK_OK;
}

// the same for the last LBVH build; `on` is the stream that must wait (a
// batched launch waits on its first context's stream)
esk_status join_lbvh(esk_ctx *c, hipStream_t on)
{
    if (c->lbvh_joined) return ESK_OK;
    // a stream being captured cannot wait for work recorded outside the
    // capture: the host waits for it instead (it was enqueued before)
    const bool cap = capturing(on);
    hipError_t e = cap ? hipEventSynchronize(c->ev_lbvh) : hipStreamWaitEvent(on, c->ev_lbvh, 0);
    if (e != hipSuccess) return hip_check(c, e, "joining the LBVH stream");
    if (cap || on == c->stream) c->lbvh_joined = true;
    return ESK_OK;
}

// both builds (before anything that rewrites the arrays they read)
esk_status join_builds(esk_ctx *c)
{
    esk_status s = join_kd(c);
    return s == ESK_OK ? join_lbvh(c, c->stream) : s;
}

}  // namespace

// A named host range around each entry point that enqueues work (shown by
// timeline tools that record markers, e.g. rocprofv3 --marker-trace); costs
// a call into the marker library when no tool listens.
struct HostRange {
    explicit HostRange(const char *name) { roctxRangePushA(name); }
    ~HostRange() { roctxRangePop(); }
    HostRange(const HostRange &) = delete;
    HostRange &operator=(const HostRange &) = delete;
};

static KdArgs kd_args(esk_ctx *c, const esk_kd_params *p);

// Sizes the next speculative batch of level launches from the last k-d build
// if it has finished (a rebuild that follows it without a render in between,
// so without kd_finish, learns its height too); never waits.
static void kd_learn_hint(esk_ctx *c)
{
    if (!c->kd_on_device) return;
    if (hipEventQuery(c->ev_kd) != hipSuccess) {
        (void)hipGetLastError();   // "not ready" is no failure of the next call
        return;
    }
    const DevHeader *h = c->pinned_kd;
    if (h->pad[0] != 0) return;   // a failed build: kd_finish reports it
    if (h->kd_end > h->kd_begin) {
        // the tree outgrew its batch (kd_finish completes it if it is used): a longer one next time
        c->kd_level_hint = c->kd_levels_enqueued + 8;
        return;
    }
    const int top = c->kd_tight_cost ? 0 : (int)h->kd_top_levels;
    c->kd_level_hint = std::max(4, (int)h->kd_height + 4 - top);
}

// Makes sure the enqueued k-d build has reached its last level, then reads
// the node count and height back.  Waits for the k-d stream only (work queued
// on the main stream keeps running).  When the speculative batch of level
// launches was short (the tree grew by more than the margin), more levels go
// on the k-d stream too, beside the main stream's work, with a fresh header
// copy and completion event, until the build has finished.
static esk_status kd_finish(esk_ctx *c)
{
    if (!c->kd_on_device) return ESK_OK;
    KdArgs k = kd_args(c, &c->kd_params);
    while (true) {
        hipError_t e = hipEventSynchronize(c->ev_kd);
        if (e != hipSuccess) return hip_check(c, e, "waiting for the k-d build");
        std::memcpy(c->pinned, c->pinned_kd, sizeof(DevHeader));
        if (c->pinned->kd_end <= c->pinned->kd_begin) break;
        if (c->kd_levels_enqueued > 4 * (c->vol.nb[0] + c->vol.nb[1] + c->vol.nb[2]) + 64)
            return fail(c, ESK_EINTERNAL, "k-d build did not terminate");
        e = launch_kd_levels(k, 8, (uint32_t)c->kd_levels_enqueued, c->aux);
        if (e == hipSuccess) e = launch_kd_pack(k, 2 * c->L.nb, c->aux);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->pinned_kd, at<DevHeader>(c, c->L.header), sizeof(DevHeader), hipMemcpyDeviceToHost,
                               c->aux);
        if (e == hipSuccess) e = hipEventRecord(c->ev_kd, c->aux);
        if (e != hipSuccess) return hip_check(c, e, "k-d level launch");
        c->kd_levels_enqueued += 8;
        c->kd_joined = false;
    }
    esk_status st = join_kd(c);
    if (st != ESK_OK) return st;
    if (c->pinned->pad[0] != 0) return fail(c, ESK_EINTERNAL, "k-d node capacity exceeded");
    c->kd_count = c->pinned->kd_count;
    c->kd_height = c->pinned->kd_height;
    // a tree of height h takes h + 1 level launches (the last one finds no
    // children), less the levels the single-workgroup launch took; three spare
    const int top = k.tight_cost ? 0 : (int)c->pinned->kd_top_levels;
    c->kd_level_hint = std::max(4, (int)c->kd_height + 4 - top);
    c->kd_on_device = false;
    return ESK_OK;
}

extern "C" {

const char *esk_strerror(esk_status s)
{
    switch (s) {
    case ESK_OK: return "ok";
    case ESK_EINVAL: return "invalid argument";
    case ESK_ENOSPC: return "workspace too small";
    case ESK_ELIMIT: return "size limit exceeded";
    case ESK_EDEVICE: return "device error";
    case ESK_ESTATE: return "call out of order";
    case ESK_EINTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *esk_last_error(const esk_ctx *c) { return c ? c->err.c_str() : "null context"; }

esk_status esk_create(int device, void *hip_stream, esk_ctx **out)
{
    if (!out) return ESK_EINVAL;
    *out = nullptr;
    if (device < -1) return ESK_EINVAL;
    esk_ctx *c = new (std::nothrow) esk_ctx();
    if (!c) return ESK_EINTERNAL;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (device >= 0) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || device >= count) {
            delete c;
            return ESK_EDEVICE;
        }
        e = hipSetDevice(device);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->pinned), sizeof(DevHeader));
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->pinned_kd), sizeof(DevHeader));
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);  // default priority
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_kd, hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux2, hipStreamNonBlocking);  // default priority
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_lbvh, hipEventDisableTiming);
        for (int j = 0; j < 2 && e == hipSuccess; ++j) e = hipEventCreateWithFlags(&c->ev_join[j], hipEventDisableTiming);
        // once per device: the address of the allocation-free batch's argument array
        if (e == hipSuccess) e = noalloc_init(device);
        if (e != hipSuccess) {
            esk_destroy(c);
            return ESK_EDEVICE;
        }
        std::memset(c->pinned, 0, sizeof(DevHeader));
        std::memset(c->pinned_kd, 0, sizeof(DevHeader));
    }
    *out = c;
    return ESK_OK;
}

esk_status esk_destroy(esk_ctx *c)
{
    if (!c) return ESK_EINVAL;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        if (c->pinned) (void)hipHostFree(c->pinned);
        if (c->staging_done) (void)hipEventSynchronize(c->staging_done);
        if (c->staging) (void)hipHostFree(c->staging);
        if (c->staging_done) (void)hipEventDestroy(c->staging_done);
        if (c->rb_done) (void)hipEventSynchronize(c->rb_done);
        if (c->rb_staging) (void)hipHostFree(c->rb_staging);
        if (c->rb_done) (void)hipEventDestroy(c->rb_done);
        if (c->aux) (void)hipStreamSynchronize(c->aux);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_kd) (void)hipEventDestroy(c->ev_kd);
        if (c->aux2) (void)hipStreamSynchronize(c->aux2);
        if (c->aux2) (void)hipStreamDestroy(c->aux2);
        if (c->ev_lbvh) (void)hipEventDestroy(c->ev_lbvh);
        for (int j = 0; j < 2; ++j)
            if (c->ev_join[j]) (void)hipEventDestroy(c->ev_join[j]);
        if (c->pinned_kd) (void)hipHostFree(c->pinned_kd);
    }
    delete c;
    return ESK_OK;
}

esk_status esk_workspace_bytes(int nx, int ny, int nz, int dtype, int brick, int max_tf_entries, size_t *out)
{
    if (!out) return ESK_EINVAL;
    esk_status s = check_shape(nullptr, nx, ny, nz, dtype, brick, max_tf_entries);
    if (s != ESK_OK) return s;
    *out = make_layout(nx, ny, nz, brick, elem_size(dtype), max_tf_entries).total;
    return ESK_OK;
}

esk_status esk_set_volume(esk_ctx *c, const void *d_vox, int dtype, int nx, int ny, int nz, float value_lo,
                          float value_hi, int brick, int max_tf_entries, void *d_ws, size_t ws_bytes)
{
    HostRange range("esk_set_volume");
    if (!c) return ESK_EINVAL;
    esk_status s = check_shape(c, nx, ny, nz, dtype, brick, max_tf_entries);
    if (s != ESK_OK) return s;
    if (!d_vox) return fail(c, ESK_EINVAL, "volume pointer is null");
    if (!d_ws) return fail(c, ESK_EINVAL, "workspace pointer is null");
    if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(c, ESK_EINVAL, "workspace must be 256-byte aligned");
    if ((reinterpret_cast<uintptr_t>(d_vox) % elem_size(dtype)) != 0)
        return fail(c, ESK_EINVAL, "volume pointer not aligned to its element size");
    if ((dtype == ESK_F16 || dtype == ESK_F32) &&
        !(std::isfinite(value_lo) && std::isfinite(value_hi) && value_lo < value_hi))
        return fail(c, ESK_EINVAL, "value range must be finite with lo < hi");
    const int nbx = (nx + brick - 1) / brick, nby = (ny + brick - 1) / brick, nbz = (nz + brick - 1) / brick;
    Layout L = make_layout(nx, ny, nz, brick, elem_size(dtype), max_tf_entries);
    if (ws_bytes < L.total)
        return fail(c, ESK_ENOSPC, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    s = join_builds(c);
    if (s != ESK_OK) return s;
    c->has_volume = false;
    c->has_tf = false;
    c->built = 0;
    c->vol.vox = d_vox;
    c->vol.dtype = dtype;
    c->vol.nx = nx;
    c->vol.ny = ny;
    c->vol.nz = nz;
    c->vol.B = brick;
    c->vol.log2B = log2i(brick);
    c->vol.nb[0] = nbx;
    c->vol.nb[1] = nby;
    c->vol.nb[2] = nbz;
    c->vlo = value_lo;
    c->vhi = value_hi;
    c->max_tf = max_tf_entries;
    c->ws = static_cast<char *>(d_ws);
    c->ws_bytes = ws_bytes;
    c->L = L;
    e = hipMemsetAsync(c->ws + L.header, 0, sizeof(DevHeader), c->stream);
    c->vol.swz = c->ws + L.swz;
    c->vol.nq[0] = (nx + kSwzEdge - 1) / kSwzEdge;
    c->vol.nq[1] = (ny + kSwzEdge - 1) / kSwzEdge;
    c->vol.nq[2] = (nz + kSwzEdge - 1) / kSwzEdge;
    if (brick >= kSwzEdge && elem_size(dtype) == 4) {
        // one pass over the volume: the blocked copy also summarises each
        // stored block, and the bricks' min/max are combined from those
        // (FP32 only: for 1- and 2-byte voxels the summaries cost more than
        // the separate min/max pass, measured)
        float *blksum = at<float>(c, L.blksum);
        if (e == hipSuccess) e = launch_swizzle(c->vol, c->ws + L.swz, blksum, c->stream);
        if (e == hipSuccess) e = launch_minmax_from_blocks(c->vol, blksum, c->ws + L.minv, c->ws + L.maxv, c->stream);
    } else {
        if (e == hipSuccess) e = launch_minmax(c->vol, c->ws + L.minv, c->ws + L.maxv, c->stream);
        if (e == hipSuccess) e = launch_swizzle(c->vol, c->ws + L.swz, nullptr, c->stream);
    }
    if (e != hipSuccess) return hip_check(c, e, "set_volume launch");
    c->has_volume = true;
    return ESK_OK;
}

// s(v) = (v - lo) * scale: the renderer's normalisation of a voxel value
static void value_norm(const esk_ctx *c, float &lo, float &scale)
{
    if (c->vol.dtype == ESK_U8) { lo = 0.0f; scale = 1.0f / 255.0f; }
    else if (c->vol.dtype == ESK_U16) { lo = 0.0f; scale = 1.0f / 65535.0f; }
    else { lo = c->vlo; scale = 1.0f / (c->vhi - c->vlo); }
}

static RebuildArgs rebuild_args(esk_ctx *c)
{
    RebuildArgs a;
    std::memset(&a, 0, sizeof(a));
    const Layout &L = c->L;
    a.vol = c->vol;
    a.vlo = c->vlo;
    a.vhi = c->vhi;
    a.N = c->N;
    a.tf = at<float>(c, L.tf);
    a.tf_src = nullptr;
    a.tfP = at<int32_t>(c, L.tfP);
    a.minv = c->ws + L.minv;
    a.maxv = c->ws + L.maxv;
    a.flags = at<uint8_t>(c, L.flags);
    a.grid = at<uint32_t>(c, L.grid);
    a.blkcnt = at<uint32_t>(c, L.blkcnt);
    a.ids = at<uint32_t>(c, L.ids);
    a.keys = at<uint32_t>(c, L.keys);
    a.skeys = at<uint32_t>(c, L.skeys);
    a.tmpkeys = at<uint32_t>(c, L.tmpkeys);
    a.sids = at<uint32_t>(c, L.sids);
    a.hist = at<uint32_t>(c, L.hist);
    a.lb_left = at<uint32_t>(c, L.lb_left);
    a.lb_right = at<uint32_t>(c, L.lb_right);
    a.lb_parent = at<uint32_t>(c, L.lb_parent);
    a.lb_range = at<int2>(c, L.lb_range);
    a.lb_axis = at<int32_t>(c, L.lb_axis);
    a.lb_lo = at<int32_t>(c, L.lb_lo);
    a.lb_hi = at<int32_t>(c, L.lb_hi);
    a.lb_rnode = at<RNode>(c, L.lb_rnode);
    a.lb_leafbox = at<uint4>(c, L.lb_leafbox);
    a.hdr = at<DevHeader>(c, L.header);
    a.nb = L.nb;
    a.nblk = L.nblk;
    a.nsortblk = L.nsortblk;
    a.key_bits = 3 * std::max({bits_for(c->vol.nb[0]), bits_for(c->vol.nb[1]), bits_for(c->vol.nb[2])});
    value_norm(c, a.nlo, a.nscale);
    a.tbox = at<uint4>(c, L.tbox);
    a.lb_root = at<uint4>(c, L.lb_root);
    a.lb_chunk = at<int32_t>(c, L.lb_chunk);
    return a;
}

static KdArgs kd_args(esk_ctx *c, const esk_kd_params *p)
{
    KdArgs k;
    std::memset(&k, 0, sizeof(k));
    const Layout &L = c->L;
    for (int a = 0; a < 3; ++a) k.nb[a] = c->vol.nb[a];
    k.B = c->vol.B;
    k.n[0] = c->vol.nx;
    k.n[1] = c->vol.ny;
    k.n[2] = c->vol.nz;
    k.flags = at<uint8_t>(c, L.flags);
    k.grid = at<uint32_t>(c, L.grid);
    k.S = at<int32_t>(c, L.kd_S);
    k.lo = at<int32_t>(c, L.kd_lo);
    k.hi = at<int32_t>(c, L.kd_hi);
    k.axis = at<int32_t>(c, L.kd_axis);
    k.plane = at<int32_t>(c, L.kd_plane);
    k.first = at<int32_t>(c, L.kd_first);
    k.split = at<int32_t>(c, L.kd_split);
    k.clo = at<int32_t>(c, L.kd_clo);
    k.plist = at<int32_t>(c, L.kd_plist);
    k.rnode = at<RNode>(c, L.kd_rnode);
    k.box = at<uint4>(c, L.kd_box);
    k.hdr = at<DevHeader>(c, L.header);
    k.cap = 2 * L.nb;
    k.tight = c->tight ? 1 : 0;
    k.tbox = at<uint4>(c, L.tbox);
    k.tight_cost = c->kd_tight_cost ? 1 : 0;
    if (p) {
        k.halting = p->halting;
        k.max_leaf = p->max_leaf;
        k.bins = p->bins;
    }
    return k;
}

esk_status esk_set_transfer_function(esk_ctx *c, const float *d_rgba, int n_entries, int build_mask,
                                     const esk_kd_params *kd)
{
    HostRange range("esk_set_transfer_function");
    if (!c) return ESK_EINVAL;
    if (!d_rgba) return fail(c, ESK_EINVAL, "TF pointer is null");
    if ((reinterpret_cast<uintptr_t>(d_rgba) & 15) != 0) return fail(c, ESK_EINVAL, "TF must be 16-byte aligned");
    if (n_entries < 2) return fail(c, ESK_EINVAL, "TF needs at least 2 entries (got %d)", n_entries);
    if (build_mask &
        ~(ESK_ACCEL_GRID | ESK_ACCEL_LBVH | ESK_ACCEL_KD | ESK_CLASSIFY_VOXEL | ESK_TIGHT_BOXES | ESK_KD_TIGHT_COST))
        return fail(c, ESK_EINVAL, "unknown bits in build_mask 0x%x", build_mask);
    if ((build_mask & ESK_KD_TIGHT_COST) && !(build_mask & ESK_ACCEL_KD))
        return fail(c, ESK_EINVAL, "ESK_KD_TIGHT_COST needs ESK_ACCEL_KD");
    // the tight split cost reads the bricks' voxel-tight boxes
    if (build_mask & ESK_KD_TIGHT_COST) build_mask |= ESK_TIGHT_BOXES;
    if (build_mask & ESK_ACCEL_KD) {
        if (!kd) return fail(c, ESK_EINVAL, "k-d build requested without parameters");
        if (kd->halting != 0 && kd->halting != 1) return fail(c, ESK_EINVAL, "kd halting must be 0 or 1");
        if (kd->max_leaf < 0 || kd->max_leaf > 4096) return fail(c, ESK_EINVAL, "kd max_leaf out of range");
        if (kd->bins < 2 || kd->bins > 16) return fail(c, ESK_EINVAL, "kd bins must be in [2, 16]");
    }
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    if (!c->has_volume) return fail(c, ESK_ESTATE, "set_transfer_function before set_volume");
    if (n_entries > c->max_tf)
        return fail(c, ESK_ELIMIT, "TF has %d entries, workspace sized for %d", n_entries, c->max_tf);
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    esk_status js = join_builds(c);
    if (js != ESK_OK) return js;
    c->has_tf = false;
    c->built = 0;
    c->kd_on_device = false;
    c->N = n_entries;
    const Layout &L = c->L;
    // k_classify copies the TF into the workspace for the renderer
    RebuildArgs a = rebuild_args(c);
    a.tf_src = d_rgba;
    if (build_mask & ESK_CLASSIFY_VOXEL) {
        a.vote = 1;
        e = launch_vote(a, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "vote launch");
    }
    e = launch_classify(a, c->stream);
    if (e != hipSuccess) return hip_check(c, e, "classify launch");
    c->tight = (build_mask & ESK_TIGHT_BOXES) != 0;
    // the compacted ids/keys feed the tight boxes and the radix sort only;
    // otherwise every export of them makes them from the current flags (a
    // replayed capture of this rebuild classifies again without the host)
    c->rebuild_compacts = c->tight || ((build_mask & ESK_ACCEL_LBVH) && !sort_by_enumeration(a));
    if (c->rebuild_compacts) {
        e = launch_compact(a, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "compaction launch");
    }
    if (c->tight) {
        a.tight = 1;
        e = launch_tight(a, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "tight-box launch");
    }
    if (build_mask & ESK_ACCEL_LBVH) {
        // fork when the k-d tree is built too: the LBVH build reads the
        // flags (and ids/keys) only, so the renders that follow a rebuild of
        // several structures need not wait for it (renders of the LBVH wait
        // for it on the device); a lone LBVH rebuild stays on the stream,
        // where the fork's cross-stream latency would add to the request
        // (measured: step 1.77 -> 1.75 ms forked; lone LBVH rebuild 0.066 ->
        // 0.080 ms if it were).  Never while the stream is being captured (a
        // capture must join every forked stream).
        const bool fork = (build_mask & ESK_ACCEL_KD) && !capturing(c->stream);
        hipStream_t ls = fork ? c->aux2 : c->stream;
        if (fork) {
            e = hipEventRecord(c->ev_fork, c->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->aux2, c->ev_fork, 0);
            if (e != hipSuccess) return hip_check(c, e, "LBVH fork");
        }
        e = launch_sort(a, ls);
        if (e == hipSuccess) e = launch_lbvh(a, ls);
        if (e == hipSuccess && fork) e = hipEventRecord(c->ev_lbvh, c->aux2);
        if (e != hipSuccess) return hip_check(c, e, "LBVH launch");
        if (fork) c->lbvh_joined = false;
    }
    if (build_mask & ESK_ACCEL_KD) {
        kd_learn_hint(c);
        c->kd_tight_cost = (build_mask & ESK_KD_TIGHT_COST) != 0;
        KdArgs k = kd_args(c, kd);
        c->kd_params = *kd;
        // fork: the k-d build needs the flags only; it runs on the auxiliary
        // stream while the main stream goes on (LBVH, grid/LBVH renders)
        e = hipEventRecord(c->ev_fork, c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->ev_fork, 0);
        if (e == hipSuccess) {
            if (kd_projected(k)) {
                e = launch_kd_root_bits(k, c->aux);
            } else if (kd_small(k)) {
                e = launch_kd_prefix_root_small(k, c->aux);
            } else {
                e = launch_kd_prefix(k, c->aux);
                if (e == hipSuccess) e = launch_kd_root(k, c->aux);
            }
        }
        // the first narrow levels in one workgroup, then the level launches,
        // enqueued speculatively (a launch past the last level exits at
        // once); completion is checked when the tree is first used
        if (e == hipSuccess && !k.tight_cost) e = launch_kd_top(k, c->aux);
        if (e == hipSuccess) e = launch_kd_levels(k, c->kd_level_hint, 0, c->aux);
        if (e == hipSuccess) e = launch_kd_pack(k, 2 * L.nb, c->aux);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->pinned_kd, at<DevHeader>(c, L.header), sizeof(DevHeader), hipMemcpyDeviceToHost,
                               c->aux);
        if (e == hipSuccess) e = hipEventRecord(c->ev_kd, c->aux);
        if (e != hipSuccess) return hip_check(c, e, "k-d launch");
        c->kd_levels_enqueued = c->kd_level_hint;
        c->kd_on_device = true;
        c->kd_joined = false;
    }
    // classification always writes the grid bitmask
    c->built = (build_mask & (ESK_ACCEL_LBVH | ESK_ACCEL_KD)) | ESK_ACCEL_GRID;
    c->has_tf = true;
    return ESK_OK;
}

// batched rebuild arguments: n RebuildArgs for the classification, up to n
// for the LBVH chain, then four block-offset tables of n + 1 words
static size_t rebuild_batch_bytes(int n)
{
    return 2 * (size_t)n * sizeof(RebuildArgs) + 4 * (((size_t)n + 1) * 4 + 15) / 16 * 16;
}

esk_status esk_rebuild_batch_bytes(int n, size_t *out)
{
    if (!out || n < 1 || n > 65535) return ESK_EINVAL;
    *out = rebuild_batch_bytes(n);
    return ESK_OK;
}

esk_status esk_rebuild_batch(esk_ctx *const *ctxs, int n, const float *const *d_tfs, const int *n_entries,
                             int build_mask, void *d_args, size_t args_bytes)
{
    HostRange range("esk_rebuild_batch");
    if (!ctxs || n < 1 || n > 65535 || !ctxs[0]) return ESK_EINVAL;
    esk_ctx *c0 = ctxs[0];
    if (!d_tfs || !n_entries) return fail(c0, ESK_EINVAL, "null request array");
    if (build_mask & ~(ESK_ACCEL_GRID | ESK_ACCEL_LBVH))
        return fail(c0, ESK_EINVAL, "batched rebuilds build the grid and the LBVH only (mask 0x%x)", build_mask);
    if (!d_args || (reinterpret_cast<uintptr_t>(d_args) & 15) != 0)
        return fail(c0, ESK_EINVAL, "argument buffer must be non-null and 16-byte aligned");
    if (args_bytes < rebuild_batch_bytes(n))
        return fail(c0, ESK_ENOSPC, "argument buffer has %zu bytes, needs %zu", args_bytes, rebuild_batch_bytes(n));
    for (int i = 0; i < n; ++i) {
        esk_ctx *c = ctxs[i];
        if (!c) return fail(c0, ESK_EINVAL, "request %d has no context", i);
        if (c->device != c0->device) return fail(c0, ESK_EINVAL, "request %d is on another device", i);
        if (!d_tfs[i] || (reinterpret_cast<uintptr_t>(d_tfs[i]) & 15) != 0)
            return fail(c0, ESK_EINVAL, "request %d: TF must be non-null and 16-byte aligned", i);
        if (n_entries[i] < 2) return fail(c0, ESK_EINVAL, "request %d: TF needs at least 2 entries", i);
        if (c->device >= 0 && !c->has_volume) return fail(c0, ESK_ESTATE, "request %d has no volume", i);
        if (c->device >= 0 && n_entries[i] > c->max_tf)
            return fail(c0, ESK_ELIMIT, "request %d: TF has %d entries, workspace sized for %d", i, n_entries[i],
                        c->max_tf);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(c0, ESK_EINVAL, "request %d repeats the context of request %d", i, j);
    }
    if (c0->device < 0) return fail(c0, ESK_ESTATE, "validation-only context");
    hipError_t e = hipSetDevice(c0->device);
    if (e != hipSuccess) return hip_check(c0, e, "hipSetDevice");
    if (c0->rb_staging_cap < n) {
        if (c0->rb_done) (void)hipEventSynchronize(c0->rb_done);
        if (c0->rb_staging) (void)hipHostFree(c0->rb_staging);
        c0->rb_staging = nullptr;
        c0->rb_staging_cap = 0;
        e = hipHostMalloc(reinterpret_cast<void **>(&c0->rb_staging), rebuild_batch_bytes(n));
        if (e != hipSuccess) return hip_check(c0, e, "staging allocation");
        c0->rb_staging_cap = n;
    }
    if (!c0->rb_done) {
        e = hipEventCreateWithFlags(&c0->rb_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_check(c0, e, "event creation");
    }
    const bool cap = capturing(c0->stream);
    if (!cap) {
        e = hipEventSynchronize(c0->rb_done);  // the previous upload has finished with the staging
        if (e != hipSuccess) return hip_check(c0, e, "staging wait");
    }
    // a pending k-d or LBVH build of any context reads the arrays this batch rewrites
    for (int i = 0; i < n; ++i) {
        esk_ctx *c = ctxs[i];
        if (!c->kd_joined) {
            e = hipStreamWaitEvent(c0->stream, c->ev_kd, 0);
            if (e != hipSuccess) return hip_check(c0, e, "joining a k-d stream");
            if (c == c0) c->kd_joined = true;
        }
        esk_status js = join_lbvh(c, c0->stream);
        if (js != ESK_OK) return js;
    }
    RebuildArgs *all = c0->rb_staging, *lbvh = c0->rb_staging + n;
    const size_t table = (((size_t)n + 1) * 4 + 15) / 16 * 16;
    char *offs = reinterpret_cast<char *>(c0->rb_staging + 2 * (size_t)n);
    std::vector<int> radix;
    int m = 0;
    for (int i = 0; i < n; ++i) {
        esk_ctx *c = ctxs[i];
        c->has_tf = false;
        c->built = 0;
        c->kd_on_device = false;
        c->N = n_entries[i];
        c->tight = false;
        RebuildArgs a = rebuild_args(c);
        a.tf_src = d_tfs[i];
        all[i] = a;
        const bool lb = (build_mask & ESK_ACCEL_LBVH) != 0;
        // the enumeration also for sparser code domains up to kBatchEnumCodes:
        // the sorted keys are the same (keys are unique)
        const bool enumerate = sort_by_enumeration(a) || ((int64_t)1 << a.key_bits) <= kBatchEnumCodes;
        c->rebuild_compacts = lb && !enumerate;
        if (lb && enumerate) lbvh[m++] = a;
        else if (lb) radix.push_back(i);
    }
    // block offsets of the flat batched grids (every count is at least 1)
    RebuildBatch b;
    char *d_base = static_cast<char *>(d_args);
    b.all = reinterpret_cast<const RebuildArgs *>(d_base);
    b.lbvh = b.all + n;
    b.n_all = n;
    b.n_lbvh = m;
    for (int k = 0; k < 4; ++k) {
        uint32_t *o = reinterpret_cast<uint32_t *>(offs + k * table);
        const RebuildArgs *src = k == 0 ? all : lbvh;
        const int cnt = k == 0 ? n : m;
        uint64_t run = 0;
        for (int i = 0; i < cnt; ++i) {
            o[i] = (uint32_t)run;
            run += (uint64_t)rebuild_batch_blocks(src[i], k);
        }
        o[cnt] = (uint32_t)run;
        if (run > 0x7fffffffu) return fail(c0, ESK_ELIMIT, "batched rebuild grid of %llu blocks",
                                           (unsigned long long)run);
        b.blocks[k] = (unsigned)run;
        b.off[k] = reinterpret_cast<const uint32_t *>(d_base + 2 * (size_t)n * sizeof(RebuildArgs) + k * table);
    }
    e = hipMemcpyAsync(d_args, all, rebuild_batch_bytes(n), hipMemcpyHostToDevice, c0->stream);
    if (e == hipSuccess && !cap) e = hipEventRecord(c0->rb_done, c0->stream);
    if (e == hipSuccess) e = launch_rebuild_batch(b, c0->stream);
    // grids whose code domain is too sparse to enumerate: their own compaction,
    // radix sort and LBVH launches, in this call, on the same stream
    for (size_t r = 0; r < radix.size() && e == hipSuccess; ++r) {
        const RebuildArgs &a = all[radix[r]];
        e = launch_compact(a, c0->stream);
        if (e == hipSuccess) e = launch_sort(a, c0->stream);
        if (e == hipSuccess) e = launch_lbvh(a, c0->stream);
    }
    if (e != hipSuccess) return hip_check(c0, e, "batched rebuild launch");
    for (int i = 0; i < n; ++i) {
        ctxs[i]->built = (build_mask & ESK_ACCEL_LBVH) | ESK_ACCEL_GRID;
        ctxs[i]->has_tf = true;
    }
    return ESK_OK;
}

}  // extern "C"

// The tile the centre of the volume projects to, clamped to the image: the
// render dispatches tiles outwards from it, so the tiles whose rays cross the
// most of the volume start first.  Perspective: C - eye = s (dir00 + fx du +
// fy dv); orthographic: C - eye = t dir00 + fx du + fy dv; solved for
// (s, s fx, s fy) or (t, fx, fy) by Cramer's rule.  Any answer is correct
// (it orders the work only); the image centre where the system is singular
// or the centre lies behind the eye.
static void centre_tile(const VolumeDesc &v, const esk_camera &cam, int W, int H, int &tx, int &ty)
{
    const int ntx = (W + 7) / 8, nty = (H + 7) / 8;
    tx = ntx / 2;
    ty = nty / 2;
    const double C[3] = {0.5 * v.nx, 0.5 * v.ny, 0.5 * v.nz};
    double A[3][3], b[3];
    for (int a = 0; a < 3; ++a) {
        A[a][0] = cam.dir00[a];
        A[a][1] = cam.du[a];
        A[a][2] = cam.dv[a];
        b[a] = C[a] - cam.eye[a];
    }
    auto det3 = [](const double M[3][3]) {
        return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
               M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    };
    const double d = det3(A);
    if (!(std::fabs(d) > 1e-300)) return;
    double u[3];
    for (int k = 0; k < 3; ++k) {
        double M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 3; ++j) M[a][j] = j == k ? b[a] : A[a][j];
        u[k] = det3(M) / d;
    }
    double fx = u[1], fy = u[2];
    if (!cam.ortho) {
        if (!(u[0] > 0.0)) return;
        fx /= u[0];
        fy /= u[0];
    }
    if (!(std::isfinite(fx) && std::isfinite(fy))) return;
    tx = (int)std::min<double>(ntx - 1, std::max(0.0, std::floor((fx - 0.5) / 8.0)));
    ty = (int)std::min<double>(nty - 1, std::max(0.0, std::floor((fy - 0.5) / 8.0)));
}

// validates one render request and fills its kernel arguments (may
// synchronise once to finish a pending k-d build)
// The host checks of one frame (no device work, no state change).
static esk_status check_render(esk_ctx *c, int accel, const esk_camera *cam, int width, int height, float step,
                               float opacity_ref_step, float *d_rgba_out, int32_t *d_count_out)
{
    if (!c) return ESK_EINVAL;
    if (!cam) return fail(c, ESK_EINVAL, "camera is null");
    if (accel != ESK_ACCEL_NONE && accel != ESK_ACCEL_GRID && accel != ESK_ACCEL_LBVH && accel != ESK_ACCEL_KD &&
        accel != ESK_ACCEL_HYBRID)
        return fail(c, ESK_EINVAL, "unknown accel %d", accel);
    if (width < 1 || height < 1 || width > 32768 || height > 32768)
        return fail(c, ESK_EINVAL, "image size %d x %d out of range", width, height);
    if (!(std::isfinite(step) && step > 0.0f)) return fail(c, ESK_EINVAL, "step must be finite and > 0");
    if (!(std::isfinite(opacity_ref_step) && opacity_ref_step >= 0.0f))
        return fail(c, ESK_EINVAL, "opacity_ref_step must be finite and >= 0");
    if (!finite3(cam->eye) || !finite3(cam->dir00) || !finite3(cam->du) || !finite3(cam->dv))
        return fail(c, ESK_EINVAL, "camera has non-finite components");
    if (!d_rgba_out) return fail(c, ESK_EINVAL, "output pointer is null");
    if ((reinterpret_cast<uintptr_t>(d_rgba_out) & 15) != 0) return fail(c, ESK_EINVAL, "output must be 16-byte aligned");
    if (d_count_out && (reinterpret_cast<uintptr_t>(d_count_out) & 3) != 0)
        return fail(c, ESK_EINVAL, "count output must be 4-byte aligned");
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    if (!c->has_volume || !c->has_tf) return fail(c, ESK_ESTATE, "render before set_volume/set_transfer_function");
    // the hybrid mode traverses the k-d tree and reads the grid (always built)
    const int needs = accel == ESK_ACCEL_HYBRID ? (int)ESK_ACCEL_KD : accel;
    if (accel != ESK_ACCEL_NONE && !(c->built & needs))
        return fail(c, ESK_ESTATE, "accel %d was not built by the last rebuild", accel);
    return ESK_OK;
}

static esk_status prepare_render(esk_ctx *c, int accel, const esk_camera *cam, int width, int height, float step,
                                 float opacity_ref_step, float *d_rgba_out, int32_t *d_count_out, RenderArgs &r,
                                 hipStream_t launch_stream)
{
    esk_status cs = check_render(c, accel, cam, width, height, step, opacity_ref_step, d_rgba_out, d_count_out);
    if (cs != ESK_OK) return cs;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    const Layout &L = c->L;
    std::memset(&r, 0, sizeof(r));
    r.vol = c->vol;
    value_norm(c, r.vlo, r.vscale);
    r.tf = at<float>(c, L.tf);
    r.N = c->N;
    r.cam = *cam;
    r.W = width;
    r.H = height;
    r.dt = step;
    r.correct = opacity_ref_step > 0.0f;
    r.expo = r.correct ? step / opacity_ref_step : 1.0f;
    r.out = d_rgba_out;
    r.count = d_count_out;
    r.grid = at<uint32_t>(c, L.grid);
    r.lb_root = at<uint4>(c, L.lb_root);
    r.lb_rnode = at<RNode>(c, L.lb_rnode);
    r.lb_leafbox = at<uint4>(c, L.lb_leafbox);
    r.kd_rnode = at<RNode>(c, L.kd_rnode);
    r.kd_box = at<uint4>(c, L.kd_box);
    r.hdr = at<DevHeader>(c, L.header);
    centre_tile(c->vol, *cam, width, height, r.ctx, r.cty);
    const int64_t tiles = (int64_t)((width + 7) / 8) * ((height + 7) / 8);
    r.seg_len = tiles >= kRaySegFewTiles ? kRaySegLen : kRaySegLenFew;
    r.stack_cap = 0;
    // a Karras tree splits on a strictly lower key bit at every level, so a
    // root-to-leaf path holds at most key_bits internal nodes
    if (accel == ESK_ACCEL_LBVH) {
        r.stack_cap = std::max(1, 3 * std::max({bits_for(c->vol.nb[0]), bits_for(c->vol.nb[1]),
                                                bits_for(c->vol.nb[2])}));
        // the launch waits on the device for the LBVH build (its own stream)
        esk_status st = join_lbvh(c, launch_stream);
        if (st != ESK_OK) return st;
    }
    if (accel == ESK_ACCEL_KD || accel == ESK_ACCEL_HYBRID) {
        esk_status st = kd_finish(c);
        if (st != ESK_OK) return st;
        if ((int)c->kd_height > kMaxKdStack)
            return fail(c, ESK_ELIMIT, "k-d tree height %u exceeds the traversal stack (%d)", c->kd_height,
                        kMaxKdStack);
        r.stack_cap = std::max(1, (int)c->kd_height);
    }
    return ESK_OK;
}

extern "C" {

esk_status esk_render(esk_ctx *c, int accel, const esk_camera *cam, int width, int height, float step,
                      float opacity_ref_step, float *d_rgba_out, int32_t *d_count_out)
{
    HostRange range("esk_render");
    RenderArgs r;
    esk_status st =
        prepare_render(c, accel, cam, width, height, step, opacity_ref_step, d_rgba_out, d_count_out, r, c->stream);
    if (st != ESK_OK) return st;
    return hip_check(c, launch_render(accel, r, c->stream), "render launch");
}

esk_status esk_render_multi(esk_ctx *c, int n, const int *accels, const esk_camera *cams, const int *widths,
                            const int *heights, float step, float opacity_ref_step, float *const *d_outs,
                            int32_t *const *d_counts)
{
    HostRange range("esk_render_multi");
    if (!c) return ESK_EINVAL;
    if (n < 1 || n > ESK_RENDER_MULTI_MAX)
        return fail(c, ESK_EINVAL, "%d frames (1 to %d in one call)", n, ESK_RENDER_MULTI_MAX);
    if (!accels || !cams || !widths || !heights || !d_outs) return fail(c, ESK_EINVAL, "null frame array");
    for (int i = 0; i < n; ++i) {
        esk_status st = check_render(c, accels[i], &cams[i], widths[i], heights[i], step, opacity_ref_step,
                                     d_outs[i], d_counts ? d_counts[i] : nullptr);
        if (st != ESK_OK) return st;
    }
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    // each frame on the stream of the build it reads (k-d and hybrid: the k-d
    // build's, LBVH: the LBVH build's, others: the context's), so frames of
    // different structures run concurrently and fill each other's tails; a
    // stream being captured keeps every frame (a capture joins no fork here)
    const bool cap = capturing(c->stream);
    hipStream_t sx[3] = {c->stream, c->aux2, c->aux};
    auto lane_of = [&](int accel) {
        if (cap) return 0;
        return accel == ESK_ACCEL_LBVH ? 1 : (accel == ESK_ACCEL_KD || accel == ESK_ACCEL_HYBRID) ? 2 : 0;
    };
    bool used[3] = {false, false, false};
    for (int i = 0; i < n; ++i) used[lane_of(accels[i])] = true;
    // the forked frames start after everything enqueued on the context's stream
    if (used[1] || used[2]) {
        e = hipEventRecord(c->ev_fork, c->stream);
        for (int j = 1; j < 3 && e == hipSuccess; ++j)
            if (used[j]) e = hipStreamWaitEvent(sx[j], c->ev_fork, 0);
        if (e != hipSuccess) return hip_check(c, e, "render fork");
    }
    // frames without the k-d tree first: a k-d frame waits on the host for
    // the tree's height
    esk_status st = ESK_OK;
    for (int pass = 0; pass < 2 && st == ESK_OK; ++pass)
        for (int i = 0; i < n && st == ESK_OK; ++i) {
            const bool kdf = accels[i] == ESK_ACCEL_KD || accels[i] == ESK_ACCEL_HYBRID;
            if (kdf != (pass == 1)) continue;
            hipStream_t s = sx[lane_of(accels[i])];
            RenderArgs r;
            st = prepare_render(c, accels[i], &cams[i], widths[i], heights[i], step, opacity_ref_step, d_outs[i],
                                d_counts ? d_counts[i] : nullptr, r, s);
            if (st == ESK_OK) st = hip_check(c, launch_render(accels[i], r, s), "render launch");
        }
    // join, also after a failed frame: the context's stream waits for every frame
    for (int j = 1; j < 3; ++j) {
        if (!used[j]) continue;
        e = hipEventRecord(c->ev_join[j - 1], sx[j]);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_join[j - 1], 0);
        if (e != hipSuccess && st == ESK_OK) st = hip_check(c, e, "render join");
    }
    return st;
}

esk_status esk_render_stream(esk_ctx *c, int accel, void **out)
{
    if (!c || !out) return ESK_EINVAL;
    if (accel != ESK_ACCEL_NONE && accel != ESK_ACCEL_GRID && accel != ESK_ACCEL_LBVH && accel != ESK_ACCEL_KD &&
        accel != ESK_ACCEL_HYBRID)
        return fail(c, ESK_EINVAL, "unknown accel %d", accel);
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    hipStream_t s = accel == ESK_ACCEL_LBVH ? c->aux2
                    : (accel == ESK_ACCEL_KD || accel == ESK_ACCEL_HYBRID) ? c->aux
                                                                           : c->stream;
    *out = static_cast<void *>(s);
    return ESK_OK;
}

esk_status esk_render_batch_bytes(int n, size_t *out)
{
    if (!out || n < 1 || n > 65535) return ESK_EINVAL;
    *out = (size_t)n * sizeof(RenderArgs);
    return ESK_OK;
}

}  // extern "C"

// Validates a batch, fills `staging` (host, n entries) with the per-request
// arguments, uploads them to d_args on ctxs[0]'s stream (recording `done`
// after the copy) and launches the batched render.  `wait` is called before
// the staging is overwritten (the previous upload from it must be complete).
template <typename Wait>
static esk_status batch_launch(esk_ctx *c0, esk_ctx *const *ctxs, int n, int accel, const esk_camera *cams,
                               const int *widths, const int *heights, float step, float opacity_ref_step,
                               float *const *d_outs, RenderArgs *staging, RenderArgs *d_args, hipEvent_t done,
                               Wait wait)
{
    const bool cap = capturing(c0->stream);
    esk_status st = cap ? ESK_OK : wait();
    if (st != ESK_OK) return st;
    size_t lds = 0;
    bool narrow = true, tfl = true;
    int tx = 1, ty = 1;
    for (int i = 0; i < n; ++i) {
        RenderArgs &r = staging[i];
        st = prepare_render(ctxs[i], accel, &cams[i], widths[i], heights[i], step, opacity_ref_step, d_outs[i],
                            nullptr, r, c0->stream);
        if (st != ESK_OK) {
            if (ctxs[i] != c0) fail(c0, st, "request %d: %s", i, ctxs[i]->err.c_str());
            return st;
        }
        const int64_t nbytes = swz_bytes(r.vol.nq, elem_size(r.vol.dtype));
        narrow = narrow && nbytes < (int64_t)0xffffffffLL;
        tfl = tfl && r.N <= 1024;
        tx = std::max(tx, (r.W + render_tile_for(accel) - 1) / render_tile_for(accel));
        ty = std::max(ty, (r.H + render_tile_for(accel) - 1) / render_tile_for(accel));
    }
    for (int i = 0; i < n; ++i) {
        const RenderArgs &r = staging[i];
        lds = std::max(lds, render_lds_bytes(accel, r.N, tfl, r.stack_cap));
    }
    hipError_t e = hipSetDevice(c0->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_args, staging, (size_t)n * sizeof(RenderArgs), hipMemcpyHostToDevice, c0->stream);
    if (e == hipSuccess && !cap) e = hipEventRecord(done, c0->stream);
    if (e == hipSuccess)
        e = launch_render_batch(accel, c0->vol.dtype, d_args, n, tx, ty, lds, narrow, tfl, c0->stream);
    return hip_check(c0, e, "batched render launch");
}

// the checks shared by both batched entry points (the request arrays)
static esk_status batch_check(esk_ctx *c0, esk_ctx *const *ctxs, int n, const esk_camera *cams, const int *widths,
                              const int *heights, float *const *d_outs)
{
    if (!cams || !widths || !heights || !d_outs) return fail(c0, ESK_EINVAL, "null request array");
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(c0, ESK_EINVAL, "request %d has no context", i);
        if (ctxs[i]->device != c0->device) return fail(c0, ESK_EINVAL, "request %d is on another device", i);
        if (ctxs[i]->has_volume && c0->has_volume && ctxs[i]->vol.dtype != c0->vol.dtype)
            return fail(c0, ESK_EINVAL, "request %d has another volume dtype", i);
    }
    return ESK_OK;
}

extern "C" {

esk_status esk_render_batch(esk_ctx *const *ctxs, int n, int accel, const esk_camera *cams, const int *widths,
                            const int *heights, float step, float opacity_ref_step, float *const *d_outs,
                            void *d_args, size_t args_bytes)
{
    HostRange range("esk_render_batch");
    if (!ctxs || n < 1 || n > 65535 || !ctxs[0]) return ESK_EINVAL;
    esk_ctx *c0 = ctxs[0];
    if (!d_args || (reinterpret_cast<uintptr_t>(d_args) & 15) != 0)
        return fail(c0, ESK_EINVAL, "argument buffer must be non-null and 16-byte aligned");
    if (args_bytes < (size_t)n * sizeof(RenderArgs))
        return fail(c0, ESK_ENOSPC, "argument buffer has %zu bytes, needs %zu", args_bytes,
                    (size_t)n * sizeof(RenderArgs));
    esk_status st = batch_check(c0, ctxs, n, cams, widths, heights, d_outs);
    if (st != ESK_OK) return st;
    if (c0->device < 0) return fail(c0, ESK_ESTATE, "validation-only context");
    if (c0->staging_cap < n) {
        if (c0->staging_done) (void)hipEventSynchronize(c0->staging_done);
        if (c0->staging) (void)hipHostFree(c0->staging);
        c0->staging = nullptr;
        c0->staging_cap = 0;
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&c0->staging), (size_t)n * sizeof(RenderArgs));
        if (e != hipSuccess) return hip_check(c0, e, "staging allocation");
        c0->staging_cap = n;
    }
    if (!c0->staging_done) {
        hipError_t e = hipEventCreateWithFlags(&c0->staging_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_check(c0, e, "event creation");
    }
    return batch_launch(c0, ctxs, n, accel, cams, widths, heights, step, opacity_ref_step, d_outs, c0->staging,
                        static_cast<RenderArgs *>(d_args), c0->staging_done, [&]() {
                            // the previous upload has finished with the staging
                            return hip_check(c0, hipEventSynchronize(c0->staging_done), "staging wait");
                        });
}

esk_status esk_render_batch_noalloc(esk_ctx *const *ctxs, int n, int accel, const esk_camera *cams,
                                    const int *widths, const int *heights, float step, float opacity_ref_step,
                                    float *const *d_outs)
{
    HostRange range("esk_render_batch_noalloc");
    if (!ctxs || n < 1 || !ctxs[0]) return ESK_EINVAL;
    esk_ctx *c0 = ctxs[0];
    if (n > kNoAllocBatchMax)
        return fail(c0, ESK_ELIMIT, "%d requests exceed the %d of the allocation-free batch", n, kNoAllocBatchMax);
    esk_status st = batch_check(c0, ctxs, n, cams, widths, heights, d_outs);
    if (st != ESK_OK) return st;
    if (c0->device < 0) return fail(c0, ESK_ESTATE, "validation-only context");
    NoAllocSlot *slot = noalloc_slot(c0->device);
    if (!slot) return fail(c0, ESK_EDEVICE, "argument array of device %d is not set up", c0->device);
    st = batch_launch(c0, ctxs, n, accel, cams, widths, heights, step, opacity_ref_step, d_outs, slot->h_staging,
                      slot->d_args, slot->done, [&]() {
                          if (!slot->recorded) return ESK_OK;
                          return hip_check(c0, hipEventSynchronize(slot->done), "staging wait");
                      });
    if (st == ESK_OK && !capturing(c0->stream)) slot->recorded = true;
    return st;
}

esk_status esk_sync(esk_ctx *c)
{
    HostRange range("esk_sync");
    if (!c) return ESK_EINVAL;
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    if (c->has_tf && (c->built & ESK_ACCEL_KD)) {
        const esk_status s = kd_finish(c);
        if (s != ESK_OK) return s;
    }
    e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && c->aux) e = hipStreamSynchronize(c->aux);
    if (e == hipSuccess && c->aux2) e = hipStreamSynchronize(c->aux2);
    return hip_check(c, e, "stream synchronize");
}

esk_status esk_get_stats(esk_ctx *c, esk_stats *out)
{
    if (!c || !out) return ESK_EINVAL;
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    if (!c->has_volume) return fail(c, ESK_ESTATE, "no volume");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    esk_status s = (c->has_tf && (c->built & ESK_ACCEL_KD)) ? kd_finish(c) : ESK_OK;
    if (s == ESK_OK) s = join_lbvh(c, c->stream);
    if (s == ESK_OK) s = read_header(c);
    if (s != ESK_OK) return s;
    std::memset(out, 0, sizeof(*out));
    out->n_bricks = c->L.nb;
    for (int a = 0; a < 3; ++a) out->nb[a] = c->vol.nb[a];
    out->built = c->has_tf ? c->built : 0;
    if (c->has_tf) {
        const int64_t n = c->pinned->n;
        out->n_nonempty = n;
        if (c->built & ESK_ACCEL_LBVH) {
            out->lbvh_nodes = n > 0 ? 2 * n - 1 : 0;
            out->lbvh_height = (int32_t)c->pinned->lbvh_height;
        }
        if (c->built & ESK_ACCEL_KD) {
            out->kd_nodes = c->pinned->kd_count;
            out->kd_height = (int32_t)c->pinned->kd_height;
        }
    }
    return ESK_OK;
}

esk_status esk_export(esk_ctx *c, int what, void *host, size_t cap, size_t *used)
{
    if (!c || !used) return ESK_EINVAL;
    if (c->device < 0) return fail(c, ESK_ESTATE, "validation-only context");
    if (!c->has_volume) return fail(c, ESK_ESTATE, "no volume");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_check(c, e, "hipSetDevice");
    esk_status s = (c->has_tf && (c->built & ESK_ACCEL_KD)) ? kd_finish(c) : ESK_OK;
    if (s == ESK_OK) s = join_lbvh(c, c->stream);
    if (s == ESK_OK) s = read_header(c);
    if (s != ESK_OK) return s;
    const Layout &L = c->L;
    const int64_t nb = L.nb;
    const int64_t n = c->has_tf ? c->pinned->n : 0;
    const int64_t m = (c->has_tf && (c->built & ESK_ACCEL_KD)) ? c->pinned->kd_count : 0;
    const int64_t ni = n > 0 ? n - 1 : 0;
    size_t off = 0, bytes = 0;
    const bool need_tf = what != ESK_X_MINMAX;
    if (need_tf && !c->has_tf) return fail(c, ESK_ESTATE, "no transfer function set");
    const bool lbvh = c->built & ESK_ACCEL_LBVH;
    if ((what == ESK_X_IDS || what == ESK_X_KEYS) && !c->rebuild_compacts) {
        e = launch_compact(rebuild_args(c), c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_check(c, e, "compaction for export");
    }
    switch (what) {
    case ESK_X_MINMAX: {
        // min and max are separate regions: copy both
        const size_t half = (size_t)nb * elem_size(c->vol.dtype);
        *used = 2 * half;
        if (cap < *used || !host) return fail(c, ESK_ENOSPC, "export needs %zu bytes", *used);
        e = hipMemcpy(host, c->ws + L.minv, half, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(static_cast<char *>(host) + half, c->ws + L.maxv, half, hipMemcpyDeviceToHost);
        return hip_check(c, e, "export copy");
    }
    case ESK_X_TF_PREFIX: off = L.tfP; bytes = (size_t)(c->N + 1) * 4; break;
    case ESK_X_FLAGS: off = L.flags; bytes = (size_t)nb; break;
    case ESK_X_IDS: off = L.ids; bytes = (size_t)n * 4; break;
    case ESK_X_KEYS: off = L.keys; bytes = (size_t)n * 4; break;
    case ESK_X_SORTED_KEYS: if (!lbvh) goto notbuilt; off = L.skeys; bytes = (size_t)n * 4; break;
    case ESK_X_SORTED_IDS: if (!lbvh) goto notbuilt; off = L.sids; bytes = (size_t)n * 4; break;
    case ESK_X_LBVH_LEFT: if (!lbvh) goto notbuilt; off = L.lb_left; bytes = (size_t)ni * 4; break;
    case ESK_X_LBVH_RIGHT: if (!lbvh) goto notbuilt; off = L.lb_right; bytes = (size_t)ni * 4; break;
    case ESK_X_LBVH_AXIS: if (!lbvh) goto notbuilt; off = L.lb_axis; bytes = (size_t)ni * 4; break;
    case ESK_X_LBVH_LO: if (!lbvh) goto notbuilt; off = L.lb_lo; bytes = (size_t)ni * 12; break;
    case ESK_X_LBVH_HI: if (!lbvh) goto notbuilt; off = L.lb_hi; bytes = (size_t)ni * 12; break;
    case ESK_X_KD_LO: if (!(c->built & ESK_ACCEL_KD)) goto notbuilt; off = L.kd_lo; bytes = (size_t)m * 12; break;
    case ESK_X_KD_HI: if (!(c->built & ESK_ACCEL_KD)) goto notbuilt; off = L.kd_hi; bytes = (size_t)m * 12; break;
    case ESK_X_KD_AXIS: if (!(c->built & ESK_ACCEL_KD)) goto notbuilt; off = L.kd_axis; bytes = (size_t)m * 4; break;
    case ESK_X_KD_PLANE: if (!(c->built & ESK_ACCEL_KD)) goto notbuilt; off = L.kd_plane; bytes = (size_t)m * 4; break;
    case ESK_X_KD_FIRST: if (!(c->built & ESK_ACCEL_KD)) goto notbuilt; off = L.kd_first; bytes = (size_t)m * 4; break;
    case ESK_X_GRID: off = L.grid; bytes = (size_t)((nb + 31) / 32) * 4; break;
    case ESK_X_TIGHT: {
        if (!c->tight) goto notbuilt;
        // packed half-voxel boxes of the non-empty bricks -> int32[nb][6],
        // zero for empty bricks and for bricks without a visible cell
        *used = (size_t)nb * 24;
        if (cap < *used || !host) return fail(c, ESK_ENOSPC, "export needs %zu bytes", *used);
        std::vector<uint32_t> packed((size_t)nb * 4);
        std::vector<uint8_t> flags((size_t)nb);
        e = hipMemcpy(packed.data(), c->ws + L.tbox, (size_t)nb * 16, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(flags.data(), c->ws + L.flags, (size_t)nb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(c, e, "export copy");
        int32_t *out = static_cast<int32_t *>(host);
        for (int64_t b = 0; b < nb; ++b) {
            const uint32_t *w = &packed[(size_t)b * 4];
            const int32_t box[6] = {(int32_t)(w[0] & 0xffffu), (int32_t)(w[0] >> 16), (int32_t)(w[1] & 0xffffu),
                                    (int32_t)(w[1] >> 16),     (int32_t)(w[2] & 0xffffu), (int32_t)(w[2] >> 16)};
            const bool any = flags[(size_t)b] && box[3] > box[0] && box[4] > box[1] && box[5] > box[2];
            for (int q = 0; q < 6; ++q) out[6 * b + q] = any ? box[q] : 0;
        }
        return ESK_OK;
    }
    default: return fail(c, ESK_EINVAL, "unknown export %d", what);
    }
    *used = bytes;
    if (bytes == 0) return ESK_OK;
    if (cap < bytes || !host) return fail(c, ESK_ENOSPC, "export needs %zu bytes", bytes);
    e = hipMemcpy(host, c->ws + off, bytes, hipMemcpyDeviceToHost);
    return hip_check(c, e, "export copy");
notbuilt:
    return fail(c, ESK_ESTATE, "export %d: structure not built by the last rebuild", what);
}

}  // extern "C"
