"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/esk.h declares, sizes workspaces, and rejects bad arguments
before touching a device (validation-only context, device = -1)."""
import ctypes
import math
import os
import re

import pytest

import paper_1912_09596_amd as esk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "esk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esk_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 11
    L = esk.lib()
    for n in names:
        assert hasattr(L, n), n


def test_workspace_bytes_and_limits():
    a = esk.workspace_bytes((64, 64, 64), esk.U8, 8, 256)
    b = esk.workspace_bytes((512, 512, 512), esk.F32, 16, 256)
    assert 0 < a < b
    # same brick grid, wider dtype -> only the min/max arrays grow
    c = esk.workspace_bytes((512, 512, 512), esk.U8, 16, 256)
    assert b > c
    out = ctypes.c_size_t()
    L = esk.lib()
    assert L.esk_workspace_bytes(64, 64, 64, esk.U8, 3, 256, ctypes.byref(out)) == esk.EINVAL
    assert L.esk_workspace_bytes(64, 64, 64, 9, 8, 256, ctypes.byref(out)) == esk.EINVAL
    assert L.esk_workspace_bytes(0, 64, 64, esk.U8, 8, 256, ctypes.byref(out)) == esk.EINVAL
    assert L.esk_workspace_bytes(64, 64, 64, esk.U8, 8, 1, ctypes.byref(out)) == esk.ELIMIT
    assert L.esk_workspace_bytes(64, 64, 64, esk.U8, 8, 4097, ctypes.byref(out)) == esk.ELIMIT
    # 1024 bricks per axis is the Morton limit
    assert L.esk_workspace_bytes(8192, 8, 8, esk.U8, 8, 256, ctypes.byref(out)) == esk.OK
    assert L.esk_workspace_bytes(8193, 8, 8, esk.U8, 8, 256, ctypes.byref(out)) == esk.ELIMIT
    # render boxes are uint16 in half-voxel units: at most 32767 voxels per axis
    assert L.esk_workspace_bytes(32767, 8, 8, esk.U8, 32, 256, ctypes.byref(out)) == esk.OK
    assert L.esk_workspace_bytes(32768, 8, 8, esk.U8, 32, 256, ctypes.byref(out)) == esk.ELIMIT
    # the renderer's blocked copy is addressed with 64-bit offsets beyond 4 GiB: no slab limit
    assert L.esk_workspace_bytes(22528, 22528, 32, esk.U8, 32, 256, ctypes.byref(out)) == esk.OK
    assert L.esk_workspace_bytes(22528, 22528, 32, esk.F32, 32, 256, ctypes.byref(out)) == esk.OK


class _VCtx:
    """validation-only context driven through the raw ABI"""

    def __init__(self):
        self.L = esk.lib()
        self.c = ctypes.c_void_p()
        assert self.L.esk_create(-1, None, ctypes.byref(self.c)) == esk.OK

    def err(self):
        return self.L.esk_last_error(self.c).decode()

    def close(self):
        assert self.L.esk_destroy(self.c) == esk.OK


FAKE = ctypes.c_void_p(0x100000)   # never dereferenced: validation-only


def test_set_volume_validation():
    v = _VCtx()
    L = v.L
    need = esk.workspace_bytes((64, 64, 64), esk.F32, 8, 256)
    sv = L.esk_set_volume
    assert sv(v.c, None, esk.F32, 64, 64, 64, 0.0, 1.0, 8, 256, FAKE, need) == esk.EINVAL
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 0.0, 1.0, 8, 256, None, need) == esk.EINVAL
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 1.0, 1.0, 8, 256, FAKE, need) == esk.EINVAL
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 0.0, math.nan, 8, 256, FAKE, need) == esk.EINVAL
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 0.0, 1.0, 12, 256, FAKE, need) == esk.EINVAL
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 0.0, 1.0, 8, 256, ctypes.c_void_p(0x100010), need) == esk.EINVAL
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 0.0, 1.0, 8, 256, FAKE, need - 1) == esk.ENOSPC
    assert "needs" in v.err()
    assert sv(v.c, FAKE, esk.F32, 64, 64, 64, 0.0, 1.0, 8, 256, FAKE, need) == esk.ESTATE
    # integer volumes ignore the value range
    need8 = esk.workspace_bytes((64, 64, 64), esk.U8, 8, 256)
    assert sv(v.c, FAKE, esk.U8, 64, 64, 64, 1.0, 1.0, 8, 256, FAKE, need8) == esk.ESTATE
    v.close()


def test_tf_and_render_validation():
    v = _VCtx()
    L = v.L
    kd = esk.KdParams(1, 0, 4)
    st = L.esk_set_transfer_function
    assert st(v.c, None, 256, esk.LBVH, None) == esk.EINVAL
    assert st(v.c, FAKE, 1, esk.LBVH, None) == esk.EINVAL
    assert st(v.c, FAKE, 256, 8, None) == esk.EINVAL
    assert st(v.c, FAKE, 256, esk.KD, None) == esk.EINVAL
    assert st(v.c, FAKE, 256, esk.KD, ctypes.byref(esk.KdParams(2, 0, 4))) == esk.EINVAL
    assert st(v.c, FAKE, 256, esk.KD, ctypes.byref(esk.KdParams(1, 0, 1))) == esk.EINVAL
    assert st(v.c, FAKE, 256, esk.KD, ctypes.byref(esk.KdParams(1, 0, 17))) == esk.EINVAL
    assert st(v.c, FAKE, 256, esk.KD | esk.LBVH, ctypes.byref(kd)) == esk.ESTATE
    # option bits: per-voxel vote and voxel-tight boxes are accepted, others not
    assert st(v.c, FAKE, 256, esk.LBVH | esk.CLASSIFY_VOXEL | esk.TIGHT_BOXES, None) == esk.ESTATE
    assert st(v.c, FAKE, 256, esk.LBVH | 0x800, None) == esk.EINVAL
    assert st(v.c, FAKE, 256, esk.LBVH | esk.KD_TIGHT_COST, None) == esk.EINVAL     # needs the k-d tree
    assert st(v.c, FAKE, 256, esk.KD | esk.KD_TIGHT_COST, ctypes.byref(kd)) == esk.ESTATE
    assert st(v.c, FAKE, 256, esk.HYBRID, None) == esk.EINVAL      # a render mode, not a structure
    cam = esk.camera_struct(dict(ortho=0, eye=[0, 0, -10], dir00=[0, 0, 1], du=[0.01, 0, 0], dv=[0, -0.01, 0]))
    r = L.esk_render
    assert r(v.c, esk.LBVH, None, 64, 64, 0.5, 1.0, FAKE, None) == esk.EINVAL
    assert r(v.c, 3, ctypes.byref(cam), 64, 64, 0.5, 1.0, FAKE, None) == esk.EINVAL
    assert r(v.c, esk.LBVH, ctypes.byref(cam), 0, 64, 0.5, 1.0, FAKE, None) == esk.EINVAL
    assert r(v.c, esk.LBVH, ctypes.byref(cam), 64, 64, 0.0, 1.0, FAKE, None) == esk.EINVAL
    assert r(v.c, esk.LBVH, ctypes.byref(cam), 64, 64, 0.5, -1.0, FAKE, None) == esk.EINVAL
    assert r(v.c, esk.LBVH, ctypes.byref(cam), 64, 64, 0.5, 1.0, None, None) == esk.EINVAL
    assert r(v.c, esk.LBVH, ctypes.byref(cam), 64, 64, 0.5, 1.0, ctypes.c_void_p(0x100004), None) == esk.EINVAL
    bad = esk.camera_struct(dict(ortho=0, eye=[0, math.inf, 0], dir00=[0, 0, 1], du=[1, 0, 0], dv=[0, 1, 0]))
    assert r(v.c, esk.LBVH, ctypes.byref(bad), 64, 64, 0.5, 1.0, FAKE, None) == esk.EINVAL
    assert r(v.c, esk.LBVH, ctypes.byref(cam), 64, 64, 0.5, 1.0, FAKE, None) == esk.ESTATE
    assert r(v.c, esk.HYBRID, ctypes.byref(cam), 64, 64, 0.5, 1.0, FAKE, None) == esk.ESTATE
    assert r(v.c, 16, ctypes.byref(cam), 64, 64, 0.5, 1.0, FAKE, None) == esk.EINVAL
    # several frames: counts, null arrays, then every frame's own checks
    m = L.esk_render_multi
    acc = (ctypes.c_int * 2)(esk.LBVH, esk.KD)
    cams = (esk.Camera * 2)(cam, cam)
    ws, hs = (ctypes.c_int * 2)(64, 64), (ctypes.c_int * 2)(64, 64)
    outs = (ctypes.c_void_p * 2)(FAKE.value, FAKE.value + 65536)
    assert m(v.c, 0, acc, cams, ws, hs, 0.5, 1.0, outs, None) == esk.EINVAL
    assert m(v.c, 9, acc, cams, ws, hs, 0.5, 1.0, outs, None) == esk.EINVAL
    assert m(v.c, 2, None, cams, ws, hs, 0.5, 1.0, outs, None) == esk.EINVAL
    assert m(v.c, 2, acc, cams, ws, hs, 0.5, 1.0, None, None) == esk.EINVAL
    assert m(v.c, 2, acc, cams, (ctypes.c_int * 2)(0, 64), hs, 0.5, 1.0, outs, None) == esk.EINVAL
    assert m(v.c, 2, (ctypes.c_int * 2)(3, esk.LBVH), cams, ws, hs, 0.5, 1.0, outs, None) == esk.EINVAL
    assert m(v.c, 2, acc, cams, ws, hs, 0.5, 1.0, outs, None) == esk.ESTATE
    assert L.esk_sync(v.c) == esk.ESTATE
    s = esk.Stats()
    assert L.esk_get_stats(v.c, ctypes.byref(s)) == esk.ESTATE
    used = ctypes.c_size_t()
    assert L.esk_export(v.c, 0, None, 0, ctypes.byref(used)) == esk.ESTATE
    v.close()


def test_batch_validation_without_a_device():
    """Both batched entry points check the request arrays and their limits on
    the host; the allocation-free one refuses more than 1024 requests."""
    v = _VCtx()
    L = v.L
    cam = esk.camera_struct(dict(ortho=0, eye=[0, 0, -10], dir00=[0, 0, 1], du=[0.01, 0, 0], dv=[0, -0.01, 0]))
    n = 2
    ctxs = (ctypes.c_void_p * n)(v.c.value, v.c.value)
    cams = (esk.Camera * n)(cam, cam)
    ws = (ctypes.c_int * n)(64, 64)
    hs = (ctypes.c_int * n)(64, 64)
    outs = (ctypes.c_void_p * n)(FAKE.value, FAKE.value)
    na = L.esk_render_batch_noalloc
    assert na(None, n, esk.LBVH, cams, ws, hs, 0.5, 1.0, outs) == esk.EINVAL
    assert na(ctxs, 0, esk.LBVH, cams, ws, hs, 0.5, 1.0, outs) == esk.EINVAL
    assert na(ctxs, n, esk.LBVH, None, ws, hs, 0.5, 1.0, outs) == esk.EINVAL
    assert na(ctxs, n, esk.LBVH, cams, ws, hs, 0.5, 1.0, None) == esk.EINVAL
    big = 1025
    bctx = (ctypes.c_void_p * big)(*([v.c.value] * big))
    bcam = (esk.Camera * big)(*([cam] * big))
    bw = (ctypes.c_int * big)(*([64] * big))
    bout = (ctypes.c_void_p * big)(*([FAKE.value] * big))
    assert na(bctx, big, esk.LBVH, bcam, bw, bw, 0.5, 1.0, bout) == esk.ELIMIT
    assert "1024" in v.err()
    assert na(ctxs, n, esk.LBVH, cams, ws, hs, 0.5, 1.0, outs) == esk.ESTATE
    assert L.esk_render_batch(ctxs, n, esk.LBVH, cams, ws, hs, 0.5, 1.0, outs, None, 0) == esk.EINVAL
    # batched rebuild: request arrays, mask, buffer, repeated contexts
    rb = L.esk_rebuild_batch
    need = ctypes.c_size_t()
    assert L.esk_rebuild_batch_bytes(2, ctypes.byref(need)) == esk.OK and need.value > 0
    assert L.esk_rebuild_batch_bytes(0, ctypes.byref(need)) == esk.EINVAL
    one = (ctypes.c_void_p * 1)(v.c.value)
    tfp = (ctypes.c_void_p * 1)(FAKE.value)
    ne = (ctypes.c_int * 1)(256)
    big_buf = ctypes.c_void_p(0x200000)
    assert rb(None, 1, tfp, ne, esk.LBVH, big_buf, 1 << 20) == esk.EINVAL
    assert rb(one, 1, None, ne, esk.LBVH, big_buf, 1 << 20) == esk.EINVAL
    assert rb(one, 1, tfp, ne, esk.KD, big_buf, 1 << 20) == esk.EINVAL
    assert rb(one, 1, tfp, ne, esk.LBVH | esk.TIGHT_BOXES, big_buf, 1 << 20) == esk.EINVAL
    assert rb(one, 1, tfp, ne, esk.LBVH, None, 1 << 20) == esk.EINVAL
    assert rb(one, 1, tfp, ne, esk.LBVH, big_buf, 16) == esk.ENOSPC
    assert rb(one, 1, (ctypes.c_void_p * 1)(0x100004), ne, esk.LBVH, big_buf, 1 << 20) == esk.EINVAL
    assert rb(one, 1, tfp, (ctypes.c_int * 1)(1), esk.LBVH, big_buf, 1 << 20) == esk.EINVAL
    two = (ctypes.c_void_p * 2)(v.c.value, v.c.value)
    assert rb(two, 2, (ctypes.c_void_p * 2)(FAKE.value, FAKE.value), (ctypes.c_int * 2)(256, 256), esk.LBVH,
              big_buf, 1 << 20) == esk.EINVAL
    assert rb(one, 1, tfp, ne, esk.LBVH, big_buf, 1 << 20) == esk.ESTATE
    assert L.esk_render_batch(ctxs, n, esk.LBVH, cams, ws, hs, 0.5, 1.0, outs, FAKE, 16) == esk.ENOSPC
    v.close()


def test_status_strings_and_null_handles():
    L = esk.lib()
    for s in (esk.OK, esk.EINVAL, esk.ENOSPC, esk.ELIMIT, esk.EDEVICE, esk.ESTATE, esk.EINTERNAL):
        assert L.esk_strerror(s)
    assert L.esk_destroy(None) == esk.EINVAL
    assert L.esk_sync(None) == esk.EINVAL
    assert L.esk_create(-2, None, ctypes.byref(ctypes.c_void_p())) == esk.EINVAL


def test_binding_rejects_bad_tensors():
    """The binding checks every tensor it hands to the library (dtype, shape,
    contiguity, device) before the call: a half-precision TF, a strided
    buffer, an undersized or host-resident image would otherwise reach the
    kernels as a wrong or wild pointer."""
    torch = pytest.importorskip("torch")
    ctx = esk.Context(-1)
    tf32 = torch.zeros((256, 4), dtype=torch.float32)
    with pytest.raises(TypeError):
        ctx.set_tf(tf32.half())                                   # 8 bytes per entry, not 16
    with pytest.raises(TypeError):
        ctx.set_tf(tf32.double())
    with pytest.raises(ValueError):
        ctx.set_tf(torch.zeros((4, 256), dtype=torch.float32).t())  # [256, 4] but strided
    with pytest.raises(ValueError):
        ctx.set_tf(torch.zeros((256, 3), dtype=torch.float32))
    with pytest.raises(ValueError):
        ctx.set_tf(tf32)                                          # host memory
    vol = torch.zeros((8, 8, 8), dtype=torch.uint8)
    with pytest.raises(ValueError):
        ctx.set_volume(vol, 8)                                    # host memory
    with pytest.raises(ValueError):
        ctx.set_volume(torch.zeros((8, 8, 16), dtype=torch.uint8)[:, :, ::2], 8)
    with pytest.raises(TypeError):
        ctx.set_volume(torch.zeros((8, 8, 8), dtype=torch.int32), 8)
    cam = dict(ortho=0, eye=[0, 0, -10], dir00=[0, 0, 1], du=[0.01, 0, 0], dv=[0, -0.01, 0])
    with pytest.raises(ValueError):
        ctx.render(cam, 16, 8, out=torch.zeros((8, 16, 4), dtype=torch.float32))      # host memory
    with pytest.raises(ValueError):
        ctx.render(cam, 16, 8, out=torch.zeros((8, 15, 4), dtype=torch.float32))      # too small
    with pytest.raises(TypeError):
        ctx.render(cam, 16, 8, out=torch.zeros((8, 16, 4), dtype=torch.float16))
    # the counts check (int32 [H, W]) is the same helper
    with pytest.raises(TypeError):
        esk._require(torch.zeros((8, 16), dtype=torch.int64), "counts", 0, torch.int32, (8, 16))
    with pytest.raises(ValueError):
        esk._require(torch.zeros((8, 17), dtype=torch.int32), "counts", 0, torch.int32, (8, 16))
    ctx.close()
