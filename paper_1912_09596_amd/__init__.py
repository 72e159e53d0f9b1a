"""MI355X-native empty-space skipping for volume ray marching.

Thin ctypes binding over ``libesk.so`` (C ABI in ``include/esk.h``): argument
marshalling only.  Every step of the hot path -- brick min/max, TF prefix
count, classification, compaction, Morton codes, radix sort, Karras LBVH,
AABB refit, binned k-d build, macrocell grid and the ray marcher -- runs in
the library's HIP kernels.  PyTorch provides device memory and the stream.

There is no fallback: if ``libesk.so`` is missing or cannot be loaded, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesk.so")

OK, EINVAL, ENOSPC, ELIMIT, EDEVICE, ESTATE, EINTERNAL = 0, -1, -2, -3, -4, -5, -6
U8, U16, F16, F32 = 0, 1, 2, 3
NONE, GRID, LBVH, KD, HYBRID = 0, 1, 2, 4, 8
CLASSIFY_VOXEL = 0x100      # build-mask bit: per-voxel vote instead of brick min/max
TIGHT_BOXES = 0x200         # build-mask bit: march LBVH/k-d leaves inside voxel-tight boxes
KD_TIGHT_COST = 0x400       # build-mask bit: k-d split cost from the voxel-tight boxes (implies TIGHT_BOXES)
ACCEL = {"none": NONE, "grid": GRID, "lbvh": LBVH, "kd": KD, "hybrid": HYBRID}
# what a rebuild must build for each render mode (the hybrid grid renders the k-d tree + grid)
BUILD = {"grid": GRID, "lbvh": LBVH, "kd": KD, "hybrid": KD}
LEAF = 0x80000000

EXPORTS = {
    "minmax": 0, "tf_prefix": 1, "flags": 2, "ids": 3, "keys": 4, "sorted_keys": 5, "sorted_ids": 6,
    "lbvh_left": 7, "lbvh_right": 8, "lbvh_axis": 9, "lbvh_lo": 10, "lbvh_hi": 11,
    "kd_lo": 12, "kd_hi": 13, "kd_axis": 14, "kd_plane": 15, "kd_first": 16, "grid": 17, "tight": 18,
}
_EXPORT_DTYPE = {
    "tf_prefix": (np.int32, 1), "flags": (np.uint8, 1), "ids": (np.uint32, 1), "keys": (np.uint32, 1),
    "sorted_keys": (np.uint32, 1), "sorted_ids": (np.uint32, 1), "lbvh_left": (np.uint32, 1),
    "lbvh_right": (np.uint32, 1), "lbvh_axis": (np.int32, 1), "lbvh_lo": (np.int32, 3),
    "lbvh_hi": (np.int32, 3), "kd_lo": (np.int32, 3), "kd_hi": (np.int32, 3), "kd_axis": (np.int32, 1),
    "kd_plane": (np.int32, 1), "kd_first": (np.int32, 1), "grid": (np.uint32, 1), "tight": (np.int32, 6),
}


class EskError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"esk status {status}: {msg}")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("ortho", ctypes.c_int32), ("eye", ctypes.c_float * 3),
                ("dir00", ctypes.c_float * 3), ("du", ctypes.c_float * 3),
                ("dv", ctypes.c_float * 3)]


class KdParams(ctypes.Structure):
    _fields_ = [("halting", ctypes.c_int32), ("max_leaf", ctypes.c_int32), ("bins", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_bricks", ctypes.c_int64), ("n_nonempty", ctypes.c_int64),
                ("lbvh_nodes", ctypes.c_int64), ("kd_nodes", ctypes.c_int64),
                ("lbvh_height", ctypes.c_int32), ("kd_height", ctypes.c_int32),
                ("nb", ctypes.c_int32 * 3), ("built", ctypes.c_int32)]


@dataclass
class Kd:
    """k-d build parameters: halting 0 = shallow (10 % of root), 1 = deep
    (8^3); max_leaf 0 = off, else the maximum-leaf-size edge; bins per axis."""
    halting: int = 1
    max_leaf: int = 0
    bins: int = 4


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libesk.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, f32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t
    L.esk_create.argtypes = [i32, P, ctypes.POINTER(P)]
    L.esk_destroy.argtypes = [P]
    L.esk_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
    L.esk_set_volume.argtypes = [P, P, i32, i32, i32, i32, f32, f32, i32, i32, P, sz]
    L.esk_set_transfer_function.argtypes = [P, P, i32, i32, ctypes.POINTER(KdParams)]
    L.esk_render.argtypes = [P, i32, ctypes.POINTER(Camera), i32, i32, f32, f32, P, P]
    L.esk_render_stream.argtypes = [P, i32, ctypes.POINTER(P)]
    L.esk_render_multi.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(Camera), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), f32, f32, ctypes.POINTER(P), ctypes.POINTER(P)]
    L.esk_sync.argtypes = [P]
    L.esk_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.esk_export.argtypes = [P, i32, P, sz, ctypes.POINTER(sz)]
    L.esk_strerror.argtypes = [i32]
    L.esk_strerror.restype = ctypes.c_char_p
    L.esk_last_error.argtypes = [P]
    L.esk_last_error.restype = ctypes.c_char_p
    L.esk_render_batch_bytes.argtypes = [i32, ctypes.POINTER(sz)]
    L.esk_render_batch.argtypes = [ctypes.POINTER(P), i32, i32, ctypes.POINTER(Camera), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), f32, f32, ctypes.POINTER(P), P, sz]
    L.esk_render_batch_noalloc.argtypes = [ctypes.POINTER(P), i32, i32, ctypes.POINTER(Camera),
                                           ctypes.POINTER(i32), ctypes.POINTER(i32), f32, f32, ctypes.POINTER(P)]
    L.esk_rebuild_batch_bytes.argtypes = [i32, ctypes.POINTER(sz)]
    L.esk_rebuild_batch.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(P), ctypes.POINTER(i32), i32, P, sz]
    for name in ("esk_create", "esk_destroy", "esk_workspace_bytes", "esk_set_volume",
                 "esk_set_transfer_function", "esk_render", "esk_render_multi", "esk_render_stream", "esk_sync",
                 "esk_get_stats", "esk_export", "esk_render_batch_bytes", "esk_render_batch", "esk_render_batch_noalloc",
                 "esk_rebuild_batch_bytes", "esk_rebuild_batch"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _dtype_code(t) -> int:
    import torch
    codes = {torch.uint8: U8, torch.uint16: U16, torch.float16: F16, torch.float32: F32}
    if t.dtype not in codes:
        raise TypeError(f"unsupported volume dtype {t.dtype}")
    return codes[t.dtype]


def _require(t, name, device, dtype=None, shape=None):
    """Raises unless tensor t has the dtype and shape the kernels read, is
    contiguous, and lives on HIP device `device` (checked before any call
    into the library: a wrong buffer would be read or written out of bounds)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device}, got {t.device}")


def workspace_bytes(dims_xyz, dtype_code: int, brick: int, max_tf: int = 4096) -> int:
    out = ctypes.c_size_t()
    st = lib().esk_workspace_bytes(int(dims_xyz[0]), int(dims_xyz[1]), int(dims_xyz[2]),
                                   dtype_code, brick, max_tf, ctypes.byref(out))
    if st != OK:
        raise EskError(st, lib().esk_strerror(st).decode())
    return out.value


def camera_struct(cam: dict) -> Camera:
    c = Camera()
    c.ortho = int(cam["ortho"])
    for name in ("eye", "dir00", "du", "dv"):
        v = np.asarray(cam[name], dtype=np.float32)
        getattr(c, name)[:] = [float(x) for x in v]
    return c


class Context:
    """One rendering context: a bound volume, its workspace, the current TF
    and the hierarchies built for it.  device=-1 gives a validation-only
    context (no GPU needed) that checks arguments and then reports ESTATE."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = lib()
        self._ctx = ctypes.c_void_p()
        self.device = device
        if device >= 0:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            handle = ctypes.c_void_p(stream.cuda_stream)
        else:
            handle = ctypes.c_void_p(0)
        self.stream = stream
        self._check(self._lib.esk_create(device, handle, ctypes.byref(self._ctx)))
        self._keep = {}

    def _on_stream(self, t):
        """A tensor allocated here on torch's current stream but used by the
        library on the context's own stream: the caching allocator must not
        hand its memory out again before that stream's work on it is done."""
        import torch
        if self.stream is not None and self.stream != torch.cuda.current_stream(self.device):
            t.record_stream(self.stream)

    def _check(self, st):
        if st != OK:
            msg = self._lib.esk_last_error(self._ctx).decode() if self._ctx else ""
            raise EskError(st, msg or self._lib.esk_strerror(st).decode())
        return st

    def close(self):
        if self._ctx:
            self._lib.esk_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ---------------------------------------------------------------
    def set_volume(self, vol, brick: int, value_range=(0.0, 1.0), max_tf: int = 1024, workspace=None):
        """vol: contiguous [nz, ny, nx] device tensor (u8/u16/f16/f32)."""
        import torch
        if not isinstance(vol, torch.Tensor) or vol.dim() != 3:
            raise ValueError("volume must be a 3-D tensor [nz, ny, nx]")
        code = _dtype_code(vol)
        _require(vol, "volume", self.device)
        nz, ny, nx = vol.shape
        need = workspace_bytes((nx, ny, nz), code, brick, max_tf)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=vol.device)
            self._on_stream(workspace)
        _require(workspace, "workspace", self.device)
        self._check(self._lib.esk_set_volume(self._ctx, ctypes.c_void_p(vol.data_ptr()), code, nx, ny, nz,
                                             float(value_range[0]), float(value_range[1]), brick, max_tf,
                                             ctypes.c_void_p(workspace.data_ptr()),
                                             workspace.numel() * workspace.element_size()))
        self._keep = {"vol": vol, "ws": workspace}
        self.dims = (nx, ny, nz)
        self.brick = brick
        self.dtype_code = code
        return self

    def set_tf(self, tf, build=("grid", "lbvh", "kd"), kd: Kd | None = None, classify: str = "minmax",
               tight: bool = False, kd_cost: str = "brick"):
        """tf: contiguous [N, 4] float32 device tensor; rebuilds the requested
        structures.  classify: "minmax" (conservative brick value ranges) or
        "voxel" (the per-voxel vote).  tight: march LBVH and k-d leaves inside
        voxel-tight boxes.  kd_cost: "brick" (brick-tight boxes) or "tight"
        (the voxel-tight boxes' unions, which also turns `tight` on)."""
        import torch
        if not isinstance(tf, torch.Tensor) or tf.dim() != 2 or tf.shape[1] != 4:
            raise ValueError("TF must be an [N, 4] float32 tensor")
        _require(tf, "TF", self.device, torch.float32)
        if classify not in ("minmax", "voxel"):
            raise ValueError("classify must be 'minmax' or 'voxel'")
        if kd_cost not in ("brick", "tight"):
            raise ValueError("kd_cost must be 'brick' or 'tight'")
        mask = (CLASSIFY_VOXEL if classify == "voxel" else 0) | (TIGHT_BOXES if tight else 0)
        if kd_cost == "tight" and "kd" in build:
            mask |= KD_TIGHT_COST
        for b in build:
            mask |= BUILD[b]
        kp = None
        if mask & KD:
            kd = kd or Kd()
            kp = KdParams(kd.halting, kd.max_leaf, kd.bins)
        self._check(self._lib.esk_set_transfer_function(self._ctx, ctypes.c_void_p(tf.data_ptr()),
                                                        tf.shape[0], mask,
                                                        ctypes.byref(kp) if kp is not None else None))
        self._keep["tf"] = tf
        return self

    def render(self, cam: dict, W: int, H: int, accel="lbvh", step=0.5, ref=1.0, out=None,
               counts=None):
        """Returns an [H, W, 4] float32 device tensor (premultiplied RGBA, row
        0 at the top).  counts: optional [H, W] int32 device tensor that
        receives the number of composited samples per pixel."""
        import torch
        if out is None:
            out = torch.empty((H, W, 4), dtype=torch.float32, device=self._keep["vol"].device)
            self._on_stream(out)
        _require(out, "out", self.device, torch.float32, (H, W, 4))
        if counts is not None:
            _require(counts, "counts", self.device, torch.int32, (H, W))
        c = camera_struct(cam)
        self._check(self._lib.esk_render(self._ctx, ACCEL[accel] if isinstance(accel, str) else int(accel),
                                         ctypes.byref(c), W, H, float(step), float(ref),
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(counts.data_ptr()) if counts is not None else None))
        return out

    def render_multi(self, frames, step=0.5, ref=1.0):
        """Several frames in one call (esk_render_multi): frames is a list of
        dicts with keys cam, W, H, accel and optionally out and counts (as in
        render); the frames of different structures render concurrently.
        Returns the list of output tensors."""
        import torch
        n = len(frames)
        if n < 1:
            raise ValueError("no frames")
        outs, cnts = [], []
        for f in frames:
            W, H = int(f["W"]), int(f["H"])
            out = f.get("out")
            if out is None:
                out = torch.empty((H, W, 4), dtype=torch.float32, device=self._keep["vol"].device)
                self._on_stream(out)
            _require(out, "out", self.device, torch.float32, (H, W, 4))
            cnt = f.get("counts")
            if cnt is not None:
                _require(cnt, "counts", self.device, torch.int32, (H, W))
            outs.append(out)
            cnts.append(cnt)
        accels = (ctypes.c_int * n)(*[ACCEL[f["accel"]] if isinstance(f["accel"], str) else int(f["accel"])
                                      for f in frames])
        cams = (Camera * n)(*[camera_struct(f["cam"]) for f in frames])
        widths = (ctypes.c_int * n)(*[int(f["W"]) for f in frames])
        heights = (ctypes.c_int * n)(*[int(f["H"]) for f in frames])
        out_ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        cnt_ptrs = (ctypes.c_void_p * n)(*[c.data_ptr() if c is not None else None for c in cnts])
        has_cnt = any(c is not None for c in cnts)
        self._check(self._lib.esk_render_multi(self._ctx, n, accels, cams, widths, heights, float(step), float(ref),
                                               out_ptrs, cnt_ptrs if has_cnt else None))
        return outs

    def render_stream(self, accel) -> int:
        """The HIP stream handle on which render_multi runs the frames of
        `accel` (for events that time them)."""
        h = ctypes.c_void_p()
        self._check(self._lib.esk_render_stream(self._ctx, ACCEL[accel] if isinstance(accel, str) else int(accel),
                                                ctypes.byref(h)))
        return h.value or 0

    def sync(self):
        self._check(self._lib.esk_sync(self._ctx))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.esk_get_stats(self._ctx, ctypes.byref(s)))
        return dict(n_bricks=s.n_bricks, n_nonempty=s.n_nonempty, lbvh_nodes=s.lbvh_nodes,
                    kd_nodes=s.kd_nodes, lbvh_height=s.lbvh_height, kd_height=s.kd_height,
                    nb=tuple(s.nb), built=s.built)

    def export(self, what: str) -> np.ndarray:
        code = EXPORTS[what]
        used = ctypes.c_size_t()
        st = self._lib.esk_export(self._ctx, code, None, 0, ctypes.byref(used))
        if st not in (OK, ENOSPC):
            self._check(st)
        if what == "minmax":
            dt = {U8: np.uint8, U16: np.uint16, F16: np.float16, F32: np.float32}[self.dtype_code]
            buf = np.empty(used.value // np.dtype(dt).itemsize, dt)
        else:
            dt, width = _EXPORT_DTYPE[what]
            buf = np.empty(used.value // np.dtype(dt).itemsize, dt)
        if used.value:
            self._check(self._lib.esk_export(self._ctx, code, buf.ctypes.data_as(ctypes.c_void_p),
                                              buf.nbytes, ctypes.byref(used)))
        if what == "minmax":
            h = buf.size // 2
            return buf[:h].copy(), buf[h:].copy()
        if width > 1:
            return buf.reshape(-1, width)
        return buf


def rebuild_batch(contexts, tfs, build=("lbvh",), args_buffer=None):
    """Sets tfs[i] on contexts[i] and rebuilds (grid and/or LBVH) for all
    requests in one launch chain on contexts[0]'s stream; each hierarchy is
    the one set_tf would build alone.  Returns the argument buffer (reusable
    once the stream has passed the call)."""
    import torch
    n = len(contexts)
    if len(tfs) != n:
        raise ValueError("contexts and tfs must have one entry per request")
    L = lib()
    need = ctypes.c_size_t()
    st = L.esk_rebuild_batch_bytes(n, ctypes.byref(need))
    if st != OK:
        raise EskError(st, "bad batch size")
    dev = contexts[0]._keep["vol"].device
    if args_buffer is None or args_buffer.numel() < need.value:
        args_buffer = torch.empty(need.value, dtype=torch.uint8, device=dev)
    _require(args_buffer, "args_buffer", contexts[0].device, torch.uint8)
    for c, tf in zip(contexts, tfs):
        if not isinstance(tf, torch.Tensor) or tf.dim() != 2 or tf.shape[1] != 4:
            raise ValueError("TF must be an [N, 4] float32 tensor")
        _require(tf, "TF", c.device, torch.float32)
    mask = 0
    for b in build:
        mask |= BUILD[b]
    ctx_arr = (ctypes.c_void_p * n)(*[c._ctx.value for c in contexts])
    tf_arr = (ctypes.c_void_p * n)(*[t.data_ptr() for t in tfs])
    n_arr = (ctypes.c_int * n)(*[int(t.shape[0]) for t in tfs])
    st = L.esk_rebuild_batch(ctx_arr, n, tf_arr, n_arr, mask, ctypes.c_void_p(args_buffer.data_ptr()),
                             args_buffer.numel())
    if st != OK:
        raise EskError(st, L.esk_last_error(contexts[0]._ctx).decode())
    for c, tf in zip(contexts, tfs):
        c._keep["tf"] = tf
    contexts[0]._keep["rebuild_args"] = args_buffer
    return args_buffer


def render_batch(contexts, cams, sizes, accel="lbvh", step=0.5, ref=1.0, outs=None, args_buffer=None):
    """Renders request i = (contexts[i], cams[i], sizes[i] = (W, H)) for all i
    in one kernel launch on contexts[0]'s stream; returns the list of [H, W, 4]
    images.  All contexts must hold volumes of one dtype on one device."""
    import torch
    n = len(contexts)
    L = lib()
    need = ctypes.c_size_t()
    st = L.esk_render_batch_bytes(n, ctypes.byref(need))
    if st != OK:
        raise EskError(st, "bad batch size")
    dev = contexts[0]._keep["vol"].device
    if args_buffer is None or args_buffer.numel() < need.value:
        args_buffer = torch.empty(need.value, dtype=torch.uint8, device=dev)
    if outs is None:
        outs = [torch.empty((h, w, 4), dtype=torch.float32, device=dev) for (w, h) in sizes]
    if not (len(cams) == n and len(sizes) == n and len(outs) == n):
        raise ValueError("contexts, cams, sizes and outs must have one entry per request")
    for c, o, (w, h) in zip(contexts, outs, sizes):
        _require(o, "out", c.device, torch.float32, (h, w, 4))
    _require(args_buffer, "args_buffer", contexts[0].device, torch.uint8)
    ctx_arr = (ctypes.c_void_p * n)(*[c._ctx.value for c in contexts])
    cam_arr = (Camera * n)(*[camera_struct(c) for c in cams])
    w_arr = (ctypes.c_int * n)(*[int(w) for (w, h) in sizes])
    h_arr = (ctypes.c_int * n)(*[int(h) for (w, h) in sizes])
    out_arr = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    code = ACCEL[accel] if isinstance(accel, str) else int(accel)
    st = L.esk_render_batch(ctx_arr, n, code, cam_arr, w_arr, h_arr, float(step), float(ref), out_arr,
                            ctypes.c_void_p(args_buffer.data_ptr()), args_buffer.numel())
    if st != OK:
        raise EskError(st, L.esk_last_error(contexts[0]._ctx).decode())
    contexts[0]._keep["batch_args"] = args_buffer
    return outs
