"""Precision: FP16 (and u16) voxel storage sampled and composited in FP32 on the
GPU, against the FP64 oracle of the FP32 source volume.  The quantisation of
the stored values is part of the error, stated per image and bounded by
4e-3 max-abs RGBA; against the oracle of the stored volume itself the bound
stays 1e-3."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_STORAGE = 4e-3
TOL_ARITH = 1e-3


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a):
    torch = _torch()
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16).copy()).view(torch.uint16).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("storage", ["f16", "u16"])
def test_reduced_precision_storage(storage):
    torch = _torch()
    import paper_1912_09596_amd as esk
    dims = (160, 144, 128)
    print(f"case: tubes {dims} stored as {storage}", flush=True)
    src = synth.tubes(dims, n_tubes=8, seed=5)                     # float32 in [0, 1]
    if storage == "f16":
        stored, lo, hi = src.astype(np.float16), 0.0, 1.0
    else:
        stored, lo, hi = np.floor(src.astype(np.float64) * 65535.0 + 0.5).astype(np.uint16), 0.0, 1.0
    tf = synth.tf_random(7, 256)
    ctx = esk.Context(0)
    ctx.set_volume(to_dev(stored), 8, (lo, hi), max_tf=256)
    ctx.set_tf(to_dev(tf), build=("grid", "lbvh", "kd"), kd=esk.Kd(1, 32, 4))
    torch.cuda.synchronize()
    # hierarchies of the stored volume are exact
    mn, mx = oracle.brick_minmax(stored, 8)
    flags = oracle.classify(mn, mx, stored.dtype, tf, lo, hi)
    assert np.array_equal(ctx.export("flags"), flags)
    errs = []
    for i, d in enumerate((synth.view_direction(1), synth.view_direction(2))):
        cam = synth.perspective(dims, 96, 80, d)
        ref_src = oracle.render(src, tf, cam, 96, 80, 0.5, 1.0, lo, hi)
        ref_stored = oracle.render(stored, tf, cam, 96, 80, 0.5, 1.0, lo, hi)
        for accel in ("none", "lbvh", "kd"):
            img = ctx.render(cam, 96, 80, accel=accel).cpu().numpy().astype(np.float64)
            e_src = np.abs(img - ref_src).max()
            e_stored = np.abs(img - ref_stored).max()
            errs.append((accel, e_src, e_stored))
            print(f"  view {i} {accel}: max|err| vs FP64 of FP32 source {e_src:.2e}, "
                  f"vs FP64 of stored volume {e_stored:.2e}", flush=True)
            assert e_stored <= TOL_ARITH
            assert e_src <= TOL_STORAGE
    assert max(e[1] for e in errs) > 0.0
