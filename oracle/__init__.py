"""CPU oracle for the empty-space-skipping hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (``paper_1912_09596_amd``)
never imports it, and it imports nothing from the product.  The arithmetic
lives in ``oracle.c`` (plain C, FP64 values, FP32 ray geometry); this module
only marshals numpy arrays into it.

Every function cites the passage of the paper (arXiv 1912.09596) it follows;
the pins that check it against facts other than itself are in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U8, U16, F16, F32 = 0, 1, 2, 3
DTYPE_CODE = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16,
              np.dtype(np.float16): F16, np.dtype(np.float32): F32}
LEAF = 0x80000000


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Camera(ctypes.Structure):
    _fields_ = [("ortho", ctypes.c_int32), ("eye", ctypes.c_float * 3),
                ("dir00", ctypes.c_float * 3), ("du", ctypes.c_float * 3),
                ("dv", ctypes.c_float * 3)]


def camera_struct(cam: dict) -> Camera:
    c = Camera()
    c.ortho = int(cam["ortho"])
    for name in ("eye", "dir00", "du", "dv"):
        v = np.asarray(cam[name], dtype=np.float32)
        getattr(c, name)[:] = [float(x) for x in v]
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        _lib.orc_brick_minmax.argtypes = [P, i32, i32, i32, i32, i32, P, P]
        _lib.orc_tf_prefix.argtypes = [P, i32, P]
        _lib.orc_classify.argtypes = [P, P, i64, i32, f32, f32, P, i32, P]
        _lib.orc_classify.restype = i64
        _lib.orc_vote.argtypes = [P, i32, i32, i32, i32, i32, f32, f32, P, i32, P]
        _lib.orc_vote.restype = i64
        _lib.orc_compact.argtypes = [P, i64, P]
        _lib.orc_compact.restype = i64
        _lib.orc_morton3.argtypes = [ctypes.c_uint32] * 3
        _lib.orc_morton3.restype = ctypes.c_uint32
        _lib.orc_morton_keys.argtypes = [P, i64, i32, i32, P]
        _lib.orc_sort_pairs.argtypes = [P, P, i64]
        _lib.orc_lbvh.argtypes = [P, P, i64, i32, i32, i32, i32, i32, i32, P, P, P, P, P]
        _lib.orc_kd.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, i32, i32, i32, i64,
                                P, P, P, P, P, P, P]
        _lib.orc_kd.restype = i64
        _lib.orc_render.argtypes = [P, i32, i32, i32, i32, f32, f32, P, i32,
                                    ctypes.POINTER(Camera), i32, i32, f32, f32, i32, P, i32,
                                    P, i64, P, P, P]
        _lib.orc_tight_boxes.argtypes = [P, i32, i32, i32, i32, f32, f32, P, i32, i32, P, P]
        _lib.orc_tight_boxes.restype = i64
        _lib.orc_ray.argtypes = [ctypes.POINTER(Camera), i32, i32, P, P]
        _lib.orc_sample.argtypes = [P, i32, i32, i32, i32, f32, f32, P, i32, P, i64, P]
        _lib.orc_threads.argtypes = []
        _lib.orc_set_threads.argtypes = [i32]
        _lib.orc_set_threads.restype = None
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check_vol(vol: np.ndarray) -> np.ndarray:
    vol = np.ascontiguousarray(vol)
    if vol.ndim != 3 or vol.dtype not in DTYPE_CODE:
        raise ValueError("volume must be a 3-D u8/u16/f16/f32 array indexed [z][y][x]")
    return vol


def brick_grid(dims_xyz, B):
    return tuple(-(-int(n) // B) for n in dims_xyz)


def brick_minmax(vol: np.ndarray, B: int):
    """a1: min/max of raw values over each brick plus a one-voxel apron (Sec. 3.1)."""
    vol = _check_vol(vol)
    nz, ny, nx = vol.shape
    nbx, nby, nbz = brick_grid((nx, ny, nz), B)
    mn = np.empty(nbx * nby * nbz, np.float64)
    mx = np.empty_like(mn)
    rc = lib().orc_brick_minmax(_p(vol), DTYPE_CODE[vol.dtype], nx, ny, nz, B, _p(mn), _p(mx))
    if rc:
        raise ValueError("orc_brick_minmax failed")
    return mn, mx


def tf_prefix(tf: np.ndarray) -> np.ndarray:
    """a2: P[i] = number of entries j < i with alpha_j > 0."""
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    P = np.empty(tf.shape[0] + 1, np.int32)
    if lib().orc_tf_prefix(_p(tf), tf.shape[0], _p(P)):
        raise ValueError("orc_tf_prefix failed")
    return P


def classify(mn, mx, dtype, tf, lo=0.0, hi=1.0) -> np.ndarray:
    """a3: brick flags (1 = may hold a visible sample) from min/max + TF prefix count."""
    mn = np.ascontiguousarray(mn, np.float64)
    mx = np.ascontiguousarray(mx, np.float64)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    flags = np.empty(mn.shape[0], np.uint8)
    code = DTYPE_CODE[np.dtype(dtype)]
    r = lib().orc_classify(_p(mn), _p(mx), mn.shape[0], code, lo, hi, _p(tf), tf.shape[0], _p(flags))
    if r < 0:
        raise ValueError("orc_classify failed")
    return flags


def vote(vol, B, tf, lo=0.0, hi=1.0) -> np.ndarray:
    """a3 variant: per-voxel vote flags (a brick's own voxels, TF lookup in FP32)."""
    vol = np.ascontiguousarray(vol)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    nz, ny, nx = vol.shape
    nb = int(np.prod(brick_grid((nx, ny, nz), B)))
    flags = np.empty(nb, np.uint8)
    code = DTYPE_CODE[vol.dtype]
    r = lib().orc_vote(_p(vol), code, nx, ny, nz, B, lo, hi, _p(tf), tf.shape[0], _p(flags))
    if r < 0:
        raise ValueError("orc_vote failed")
    return flags


def tight_boxes(vol, B, tf, flags, lo=0.0, hi=1.0) -> np.ndarray:
    """Voxel-tight box of every brick, (nb, 6) int32 in half-voxel units
    (lo2 x, y, z, hi2 x, y, z; the box is [lo2/2, hi2/2)): the bounding box
    of its potentially visible trilinear cells; all zero when empty."""
    vol = np.ascontiguousarray(vol)
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    flags = np.ascontiguousarray(flags, np.uint8)
    nz, ny, nx = vol.shape
    boxes = np.empty((flags.shape[0], 6), np.int32)
    r = lib().orc_tight_boxes(_p(vol), DTYPE_CODE[vol.dtype], nx, ny, nz, lo, hi, _p(tf), tf.shape[0], B,
                              _p(flags), _p(boxes))
    if r < 0:
        raise ValueError("orc_tight_boxes failed")
    return boxes


def compact(flags) -> np.ndarray:
    """a4: ids of flagged bricks, ascending."""
    flags = np.ascontiguousarray(flags, np.uint8)
    ids = np.empty(max(1, flags.shape[0]), np.uint32)
    n = lib().orc_compact(_p(flags), flags.shape[0], _p(ids))
    return ids[:n].copy()


def morton3(x: int, y: int, z: int) -> int:
    """a5: 30-bit Morton code, x -> bit 3i+2, y -> 3i+1, z -> 3i."""
    return int(lib().orc_morton3(x, y, z))


def morton_keys(ids, nbx, nby) -> np.ndarray:
    ids = np.ascontiguousarray(ids, np.uint32)
    keys = np.empty(max(1, ids.shape[0]), np.uint32)
    lib().orc_morton_keys(_p(ids), ids.shape[0], nbx, nby, _p(keys))
    return keys[:ids.shape[0]].copy()


def sort_pairs(keys, ids):
    """a6: (key, id) pairs ordered by key."""
    k = np.array(keys, np.uint32)
    i = np.array(ids, np.uint32)
    if lib().orc_sort_pairs(_p(k), _p(i), k.shape[0]):
        raise MemoryError
    return k, i


def lbvh(sorted_keys, sorted_ids, B, dims_xyz):
    """a7+a8: Karras-numbered radix tree over sorted keys, with internal AABBs
    (voxel units, half-open) and the height in levels (Sec. 3.1)."""
    k = np.ascontiguousarray(sorted_keys, np.uint32)
    i = np.ascontiguousarray(sorted_ids, np.uint32)
    n = k.shape[0]
    nx, ny, nz = dims_xyz
    nbx, nby, _ = brick_grid(dims_xyz, B)
    m = max(1, n - 1)
    left = np.zeros(m, np.uint32)
    right = np.zeros(m, np.uint32)
    axis = np.zeros(m, np.int32)
    lo = np.zeros((m, 3), np.int32)
    hi = np.zeros((m, 3), np.int32)
    h = lib().orc_lbvh(_p(k), _p(i), n, nbx, nby, B, nx, ny, nz, _p(left), _p(right), _p(axis),
                       _p(lo), _p(hi))
    m = max(0, n - 1)
    return dict(keys=k, ids=i, left=left[:m], right=right[:m], axis=axis[:m], lo=lo[:m],
                hi=hi[:m], height=int(h))


def kd(flags, B, dims_xyz, halting=1, max_leaf=0, bins=4, tight_boxes=None):
    """a10: binned k-d tree over brick occupancy, BFS order (Sec. 3.2, 4.3).
    tight_boxes: None for the brick-granular cost, else the (nb, 6) voxel-
    tight boxes of tight_boxes(): the split cost and every volume the build
    compares use the unions of those boxes (Sec. 3.2.2)."""
    flags = np.ascontiguousarray(flags, np.uint8)
    nx, ny, nz = dims_xyz
    nbx, nby, nbz = brick_grid(dims_xyz, B)
    cap = max(1, 2 * int(flags.sum()) - 1)
    lo = np.zeros((cap, 3), np.int32)
    hi = np.zeros((cap, 3), np.int32)
    axis = np.zeros(cap, np.int32)
    plane = np.zeros(cap, np.int32)
    first = np.zeros(cap, np.int32)
    height = np.zeros(1, np.int32)
    tb = None if tight_boxes is None else np.ascontiguousarray(tight_boxes, np.int32).reshape(-1, 6)
    if tb is not None and tb.shape[0] != flags.shape[0]:
        raise ValueError("tight_boxes needs one box per brick")
    n = lib().orc_kd(_p(flags), nbx, nby, nbz, B, nx, ny, nz, halting, max_leaf, bins, cap,
                     _p(lo), _p(hi), _p(axis), _p(plane), _p(first), _p(height),
                     _p(tb) if tb is not None else None)
    if n < 0:
        raise RuntimeError("orc_kd: capacity exceeded")
    return dict(lo=lo[:n], hi=hi[:n], axis=axis[:n], plane=plane[:n], first_child=first[:n],
                height=int(height[0]))


def render(vol, tf, cam: dict, W, H, dt=0.5, ref=1.0, lo=0.0, hi=1.0, mode=0, flags=None, B=0,
           pixels=None, with_counts=False, boxes=None):
    """a11-a14: FP64 image of the full march (mode 0), of the brick-skipping
    march (mode 1: samples of flagged bricks) or of the tight-box march
    (mode 2: samples inside their flagged brick's tight box, `boxes` as
    returned by tight_boxes).  pixels: optional (n,2) int array of (x,y) to
    render one by one; returns (n,4) then, else (H,W,4)."""
    vol = _check_vol(vol)
    nz, ny, nx = vol.shape
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    c = camera_struct(cam)
    if pixels is not None:
        pix = np.ascontiguousarray(pixels, np.int32).reshape(-1, 2)
        out = np.zeros((pix.shape[0], 4), np.float64)
        npix = pix.shape[0]
        pp = _p(pix)
    else:
        out = np.zeros((H, W, 4), np.float64)
        npix = 0
        pp = None
    counts = np.zeros(out.shape[:-1], np.int64)
    fl = np.ascontiguousarray(flags, np.uint8) if flags is not None else None
    rc = lib().orc_render(_p(vol), DTYPE_CODE[vol.dtype], nx, ny, nz, lo, hi, _p(tf), tf.shape[0],
                          ctypes.byref(c), W, H, dt, ref, mode, _p(fl) if fl is not None else None,
                          B, pp, npix, _p(out), _p(counts),
                          _p(np.ascontiguousarray(boxes, np.int32)) if boxes is not None else None)
    if rc:
        raise ValueError("orc_render failed")
    return (out, counts) if with_counts else out


def ray(cam: dict, px: int, py: int):
    """a11: the FP32 ray (origin, unit direction) of pixel (px, py)."""
    c = camera_struct(cam)
    o = np.zeros(3, np.float32)
    d = np.zeros(3, np.float32)
    lib().orc_ray(ctypes.byref(c), px, py, _p(o), _p(d))
    return o, d


def sample(vol, tf, points, lo=0.0, hi=1.0):
    """Post-classified RGBA (before opacity correction) at FP32 points (n,3),
    given as (x, y, z) in voxel units (Sec. 4.1: post-classification)."""
    vol = _check_vol(vol)
    nz, ny, nx = vol.shape
    tf = np.ascontiguousarray(tf, dtype=np.float32)
    pts = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    out = np.zeros((pts.shape[0], 4), np.float64)
    lib().orc_sample(_p(vol), DTYPE_CODE[vol.dtype], nx, ny, nz, lo, hi, _p(tf), tf.shape[0],
                     _p(pts), pts.shape[0], _p(out))
    return out
